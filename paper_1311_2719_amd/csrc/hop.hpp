// The staggered hop sum (the inner loop of the paper's matrix-vector routine,
// Sec. 3) as device building blocks shared by the standalone D_slash and the
// fused CG kernels.
//
// One output site is processed by LPS lanes (LPS = 1, 2, 4, 8) of one
// wavefront.  Lanes are numbered sub-major: lane = sub * (64/LPS) + i, so the
// lanes that share `sub` take 64/LPS consecutive sites and every load they
// issue is unit-stride.  Lane `sub` takes the directions d = sub, sub + LPS,
// ... and the partial sums of a site are combined with cross-lane shuffles
// (xor 32, 16, 8).  R right-hand sides that share the gauge field are processed
// together so that each link entry is loaded once for all of them.
#pragma once

#include "stag_types.hpp"

namespace stag {

// Map the hardware block index to a logical one so that each XCD (blocks are
// dealt to the 8 XCDs round-robin) works on one contiguous range of sites:
// neighbour spinors of a range then stay in that XCD's L2.
__device__ __forceinline__ int logical_block(int b, int nblocks, int remap)
{
    if (!remap)
        return b;
    const int q = nblocks >> 3, rem = nblocks & 7;
    const int xcd = b & 7, i = b >> 3;
    return xcd * q + (xcd < rem ? xcd : rem) + i;
}

// Site and lane-within-site of global thread gt (blocks are whole wavefronts).
template <int LPS> __device__ __forceinline__ void site_of_thread(int gt, int &s, int &sub)
{
    constexpr int SPW = 64 / LPS;  // sites per wavefront
    const int lane = gt & 63;
    sub = lane / SPW;
    s = (gt >> 6) * SPW + (lane % SPW);
}

template <int LPS, typename T> __device__ __forceinline__ T lane_sum(T v)
{
#pragma unroll
    for (int o = 32; o >= 64 / LPS; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// acc[r][a] += sum over this lane's directions of L_d(s)[a][b] in_r(n_d(s))[b],
// then summed over the LPS lanes of the site.  load(r, n, chi) fetches the
// input colour vector of right-hand side r at neighbour site n.  Every
// right-hand side of the tile is computed, so load must stay in bounds for
// each r; callers discard the sums of systems they do not update (a
// per-system test inside the direction loop would split it into blocks that
// each wait for their loads).  LEAN keeps
// the direction loop rolled (LEAN_UNROLL directions' loads in flight at a
// time), for rarely taken paths that must not raise the register budget of
// the kernel they live in.  ROWS = 3: all 9 link entries are stored; ROWS = 2:
// rows 0 and 1 are stored and row 2 is rebuilt in registers.
template <class P, int LPS, int R, class Load, bool LEAN, int ROWS, int LEAN_UNROLL, bool TABLES>
__device__ __forceinline__ void hop_accumulate_impl(const Geom &g, const typename P::link_t *__restrict__ links,
                                                    const int32_t *__restrict__ nbr, int p_out, int s, int sub,
                                                    cplx<typename P::real> (*acc)[3], Load load)
{
    using real = typename P::real;
    static_assert(ROWS == 2 || ROWS == 3, "links are stored with 2 or 3 rows");
    SiteCoord c;
    if constexpr (!TABLES || ROWS == 2)
        c = decode_site(g, p_out, s);
    auto one_direction = [&](int j) {
        const int d = sub + j * LPS;
        int n;
        if constexpr (TABLES)
            n = nbr[(int64_t)d * g.Vh + s];
        else
            n = neighbour(g, c, s, d);
        cplx<real> U[9];
        const typename P::link_t *lp = links + link_offset(g.Vh, d, 0, s);
#pragma unroll
        for (int k = 0; k < 3 * ROWS; ++k)
            U[k] = P::load_link(lp + (int64_t)k * 8 * g.Vh);
        if constexpr (ROWS == 2)
            third_row(U, folded_negative(g, c, d) ? real(-2) : real(2));
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cplx<real> chi[3];
            load(r, n, chi);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    cmac(acc[r][a], U[a * 3 + b], chi[b]);
        }
    };
    if constexpr (LEAN) {
#pragma unroll LEAN_UNROLL
        for (int j = 0; j < 8 / LPS; ++j)
            one_direction(j);
    } else {
#pragma unroll
        for (int j = 0; j < 8 / LPS; ++j)
            one_direction(j);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc[r][a].re = lane_sum<LPS>(acc[r][a].re);
            acc[r][a].im = lane_sum<LPS>(acc[r][a].im);
        }
}

// The hop with the neighbour source (tables or coordinates) decided once,
// outside the direction loop: a choice inside it would merge the table load
// and the computed index into one register, and the wait for that load would
// drain every load in flight at each direction.
template <class P, int LPS, int R, class Load, bool LEAN = false, int ROWS = 3, int LEAN_UNROLL = 1>
__device__ __forceinline__ void hop_accumulate(const Geom &g, const typename P::link_t *__restrict__ links,
                                               const int32_t *__restrict__ nbr, int p_out, int s, int sub,
                                               cplx<typename P::real> (*acc)[3], Load load)
{
    if (nbr)
        hop_accumulate_impl<P, LPS, R, Load, LEAN, ROWS, LEAN_UNROLL, true>(g, links, nbr, p_out, s, sub, acc,
                                                                             load);
    else
        hop_accumulate_impl<P, LPS, R, Load, LEAN, ROWS, LEAN_UNROLL, false>(g, links, nbr, p_out, s, sub, acc,
                                                                              load);
}

// Colour c of an output site is written / reduced by lane (c mod LPS).
template <int LPS> __device__ __forceinline__ bool owns_colour(int sub, int c) { return (c % LPS) == sub; }

// ---- block reductions (deterministic: fixed shuffle tree, fixed LDS order) ----

// A double moved across lanes by a DPP control (two 32-bit moves).
template <int CTRL> __device__ __forceinline__ double dpp_move(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 64 lanes of a wavefront (every lane must be active), returned
// in every lane.  Within each row of 16 lanes the sum is formed by DPP moves
// (pairs, quads, half-row mirror, row mirror: no LDS round trips), then the
// four row sums are added in a fixed order.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_move<0xb1>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4e>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum v[r] over the block; thread r (< R) receives the total of column r.
// lds must hold R * (blockDim.x / 64) doubles.
template <int R> __device__ __forceinline__ void block_sum_multi(double (&v)[R], double *lds, double &out)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double t = wave_sum(v[r]);
        if (lane == 0)
            lds[r * nw + w] = t;
    }
    __syncthreads();
    out = 0.0;
    if (threadIdx.x < R)
        for (int i = 0; i < nw; ++i)
            out += lds[threadIdx.x * nw + i];
    __syncthreads();
}

// Total of partials[0 .. n) in a fixed order (a strided sum per thread, then
// the block tree); valid in thread 0.
__device__ __forceinline__ double reduce_partials(const double *partials, int n, double *lds)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        v += partials[i];
    double arr[1] = {v};
    double out;
    block_sum_multi<1>(arr, lds, out);
    return out;
}

}  // namespace stag
