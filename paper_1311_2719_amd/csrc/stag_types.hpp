// Device-side types shared by the HIP kernels of libstagcg.
//
// Storage formats (structure-of-arrays over the checkerboard index of one
// parity, so lanes that take consecutive sites touch consecutive addresses):
//   links   per parity [entry 9][site tile Vh/8][dir 8][site 8] of a complex
//           type: each (entry, tile) is a contiguous 8 x 8 block, so a
//           wavefront reading one entry for 64 consecutive sites and one
//           direction, or for 8 sites and all 8 directions, touches whole
//           cache lines either way.  Dir 0..3 are the forward links
//           W_mu(x) = 1/2 eta_mu(x) s_fwd(x) U_mu(x), dir 4..7 the backward
//           links B_mu(x) = -1/2 eta_mu(x) s_bwd(x) U_mu(x-mu)^dagger, both stored
//           at the site x that uses them; s_fwd / s_bwd are the t-boundary
//           signs.  With these, (D chi)(x) = sum_d L_d(x) chi(n_d(x)),
//           n_d = x+mu (d < 4) or x-mu (d >= 4).  Vh is a multiple of 8
//           because every extent is even.
//           Two-row form (fields whose links are special unitary): only
//           entries 0..5 (rows 0 and 1) are stored.  Every stored matrix is
//           c V with V in SU(3) and c = +-1/2, so row 2 = conj(row0 x row1) / c,
//           with the sign of c recomputed from the site's coordinates.
//   spinors FP64 / FP32: [colour 3][Vh] of complex; FP16: one 16-byte record
//           per site (3 half2 colours scaled by 1/norm, and the FP32 norm =
//           largest |component| of the site).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stagcg.h"

namespace stag {

typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt2 __attribute__((ext_vector_type(2)));
typedef _Float16 hlf2 __attribute__((ext_vector_type(2)));

struct __attribute__((aligned(16))) HalfSpinor {
    hlf2 c[3];
    float norm;
};
static_assert(sizeof(HalfSpinor) == 16, "half spinor record must be 16 bytes");

// Lattice geometry of one parity in checkerboard order.
struct Geom {
    int32_t L[4];
    int32_t Lxh;  // Lx / 2
    int32_t Vh;   // sites per parity
    int32_t sy;   // checkerboard stride of one step in y: Lxh
    int32_t sz;   // ... in z: Lxh * Ly
    int32_t st;   // ... in t: Lxh * Ly * Lz
    int32_t tap;  // 1: antiperiodic in t (the sign is folded into the links)
};

inline Geom make_geom(const int32_t d[4])
{
    Geom g;
    for (int i = 0; i < 4; ++i)
        g.L[i] = d[i];
    g.Lxh = d[0] / 2;
    g.Vh = (int32_t)((int64_t)d[0] * d[1] * d[2] * d[3] / 2);
    g.sy = g.Lxh;
    g.sz = g.Lxh * d[1];
    g.st = g.Lxh * d[1] * d[2];
    g.tap = 0;
    return g;
}

// Link entries per output parity: 8 directions x (3 x rows) complex per site.
__host__ __device__ __forceinline__ int64_t link_parity_entries(int rows, int Vh)
{
    return (int64_t)24 * rows * Vh;
}

// Offset of link entry k of direction d at checkerboard site s, within one parity.
__host__ __device__ __forceinline__ int64_t link_offset(int Vh, int d, int k, int s)
{
    return (int64_t)k * 8 * Vh + (int64_t)(s >> 3) * 64 + d * 8 + (s & 7);
}

struct SiteCoord {
    int x, y, z, t;
    int base;  // checkerboard index of (x = 0 or 1, y, z, t)
};

// Coordinates of checkerboard site s of parity p.
__device__ __forceinline__ SiteCoord decode_site(const Geom &g, int p, int s)
{
    SiteCoord c;
    const int xh = s % g.Lxh;
    int r = s / g.Lxh;
    c.y = r % g.L[1];
    r /= g.L[1];
    c.z = r % g.L[2];
    c.t = r / g.L[2];
    c.x = 2 * xh + ((p + c.y + c.z + c.t) & 1);
    c.base = s - xh;
    return c;
}

// True when the real factor folded into link d of the site with coordinates
// c is negative: eta_mu(x), the minus of a backward link and the sign of a hop
// across the t boundary of an antiperiodic field (the rule the gauge
// preparation applies).
__device__ __forceinline__ bool folded_negative(const Geom &g, const SiteCoord &c, int d)
{
    // every field is read before any choice is made, so the choices below
    // select between values and never become a per-lane indexed memory access
    const int cx = c.x, cy = c.y, cz = c.z, ct = c.t, tap = g.tap, Lt = g.L[3];
    const int mu = d & 3;
    const int esum = (mu > 0 ? cx : 0) + (mu > 1 ? cy : 0) + (mu > 2 ? cz : 0);
    const bool back = d >= 4;
    const bool wrap = tap && mu == 3 && (back ? ct == 0 : ct == Lt - 1);
    return ((esum & 1) != 0) != (back != wrap);
}

// Checkerboard index (in the other parity) of neighbour d of site s:
// d = 0..3 forward in x,y,z,t; d = 4..7 backward.  Written with selects on
// values only, so lanes of one wavefront that take different directions
// neither diverge nor index memory by lane.
__device__ __forceinline__ int neighbour(const Geom &g, const SiteCoord &c, int s, int d)
{
    const int cx = c.x, cy = c.y, cz = c.z, ct = c.t, base = c.base;
    const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3], sy = g.sy, sz = g.sz, st_t = g.st;
    const int mu = d & 3;
    const bool fwd = d < 4;
    const int xn = fwd ? (cx + 1 == L0 ? 0 : cx + 1) : (cx == 0 ? L0 - 1 : cx - 1);
    const int nx = base + (xn >> 1);
    const int co = mu == 1 ? cy : (mu == 2 ? cz : ct);
    const int L = mu == 1 ? L1 : (mu == 2 ? L2 : L3);
    const int st = mu == 1 ? sy : (mu == 2 ? sz : st_t);
    const int nf = co + 1 == L ? s - (L - 1) * st : s + st;
    const int nb = co == 0 ? s + (L - 1) * st : s - st;
    return mu == 0 ? nx : (fwd ? nf : nb);
}

// ---- complex arithmetic in the compute type --------------------------------

template <typename T> struct cplx {
    T re, im;
};

template <typename T> __device__ __forceinline__ cplx<T> czero() { return {T(0), T(0)}; }

// acc += a * b
template <typename T>
__device__ __forceinline__ void cmac(cplx<T> &acc, const cplx<T> &a, const cplx<T> &b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}

// Row 2 of W = c V (V special unitary, c real) from rows 0 and 1 (entries
// U[0..5], row-major): W_2 = conj(W_0 x W_1) / c; inv_c = 1 / c.
template <typename T> __device__ __forceinline__ void third_row(cplx<T> (&U)[9], T inv_c)
{
    // z = a_i b_j - a_j b_i for rows a = U[0..2], b = U[3..5]
    auto cross = [&](int i, int j) {
        cplx<T> z;
        z.re = U[i].re * U[3 + j].re - U[i].im * U[3 + j].im - (U[j].re * U[3 + i].re - U[j].im * U[3 + i].im);
        z.im = U[i].re * U[3 + j].im + U[i].im * U[3 + j].re - (U[j].re * U[3 + i].im + U[j].im * U[3 + i].re);
        return z;
    };
    const cplx<T> z0 = cross(1, 2), z1 = cross(2, 0), z2 = cross(0, 1);
    U[6] = {z0.re * inv_c, -z0.im * inv_c};
    U[7] = {z1.re * inv_c, -z1.im * inv_c};
    U[8] = {z2.re * inv_c, -z2.im * inv_c};
}

// ---- precision traits --------------------------------------------------------
//
// Each precision defines the link storage type, the spinor storage format used
// for vectors that D gathers (p, ap), the compute type, and load/store helpers.

struct PrecF64 {
    using real = double;
    using link_t = dbl2;
    static constexpr int id = 0;
    // spinor storage: [3][Vh] dbl2
    using spin_store = dbl2;
    static __device__ __forceinline__ cplx<real> load_link(const link_t *p)
    {
        const dbl2 v = *p;
        return {v.x, v.y};
    }
    static __device__ __forceinline__ void load_spinor(const void *base, int Vh, int s, cplx<real> out[3])
    {
        const dbl2 *b = (const dbl2 *)base;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dbl2 v = b[(int64_t)c * Vh + s];
            out[c] = {v.x, v.y};
        }
    }
    static __device__ __forceinline__ void store_spinor(void *base, int Vh, int s, const cplx<real> v[3])
    {
        dbl2 *b = (dbl2 *)base;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            b[(int64_t)c * Vh + s] = dbl2{v[c].re, v[c].im};
    }
    static constexpr size_t spinor_bytes = 48;  // per site
    static constexpr size_t link_bytes = 16;     // per complex entry
};

// FP64 with non-temporal link loads, for fields whose FP64 links do not fit
// the 256 MB Infinity Cache.  A kernel reads each link once and never again
// while it runs; non-temporal loads keep the links from evicting the
// gathered vectors, which every site reads eight times (32^4 D_slash:
// 170 -> 152 us, FP64 CG 4.14 -> 4.80 solves/s).  Where the links do fit,
// the cache serves them across the CG's kernels and plain loads are faster
// (16^4 CG: 238 against 213 solves/s; 24^4: 22.6 against 21.6).  The FP32
// and FP16 tiles measured slower with them at every size.
struct PrecF64NT : PrecF64 {
    static __device__ __forceinline__ cplx<real> load_link(const link_t *p)
    {
        const dbl2 v = __builtin_nontemporal_load(p);
        return {v.x, v.y};
    }
};

struct PrecF32 {
    using real = float;
    using link_t = flt2;
    static constexpr int id = 1;
    static __device__ __forceinline__ cplx<real> load_link(const link_t *p)
    {
        flt2 v = *p;
        return {v.x, v.y};
    }
    static __device__ __forceinline__ void load_spinor(const void *base, int Vh, int s, cplx<real> out[3])
    {
        const flt2 *b = (const flt2 *)base;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            flt2 v = b[(int64_t)c * Vh + s];
            out[c] = {v.x, v.y};
        }
    }
    static __device__ __forceinline__ void store_spinor(void *base, int Vh, int s, const cplx<real> v[3])
    {
        flt2 *b = (flt2 *)base;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            b[(int64_t)c * Vh + s] = flt2{v[c].re, v[c].im};
    }
    static constexpr size_t spinor_bytes = 24;
    static constexpr size_t link_bytes = 8;
};

struct PrecF16 {
    using real = float;
    using link_t = hlf2;
    static constexpr int id = 2;
    static __device__ __forceinline__ cplx<real> load_link(const link_t *p)
    {
        hlf2 v = *p;
        return {(float)v.x, (float)v.y};
    }
    static __device__ __forceinline__ void decode(const HalfSpinor &h, cplx<real> out[3])
    {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            out[c] = {(float)h.c[c].x * h.norm, (float)h.c[c].y * h.norm};
    }
    static __device__ __forceinline__ HalfSpinor encode(const cplx<real> v[3])
    {
        float m = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
        HalfSpinor h;
        const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            h.c[c] = hlf2{(_Float16)(v[c].re * inv), (_Float16)(v[c].im * inv)};
        h.norm = m;
        return h;
    }
    static __device__ __forceinline__ void load_spinor(const void *base, int, int s, cplx<real> out[3])
    {
        decode(((const HalfSpinor *)base)[s], out);
    }
    static __device__ __forceinline__ void store_spinor(void *base, int, int s, const cplx<real> v[3])
    {
        ((HalfSpinor *)base)[s] = encode(v);
    }
    // store v and replace it by the value a later load_spinor returns
    // (for norms of stored vectors, without reading the store back)
    static __device__ __forceinline__ void store_spinor_read_back(void *base, int, int s, cplx<real> v[3])
    {
        const HalfSpinor h = encode(v);
        ((HalfSpinor *)base)[s] = h;
        decode(h, v);
    }
    static constexpr size_t spinor_bytes = 16;
    static constexpr size_t link_bytes = 4;
};

// Bytes per site of one stored spinor / one link field entry, per precision id.
inline size_t spinor_bytes_of(int prec) { return prec == 0 ? 48 : prec == 1 ? 24 : 16; }
inline size_t link_entry_bytes_of(int prec) { return prec == 0 ? 16 : prec == 1 ? 8 : 4; }

}  // namespace stag
