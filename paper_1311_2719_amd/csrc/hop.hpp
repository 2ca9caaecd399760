// The staggered hop sum (the inner loop of the paper's matrix-vector routine,
// Sec. 3) as device building blocks shared by the standalone D_slash and the
// fused CG kernels.
//
// One output site is processed by LPS lanes (LPS = 1, 2, 4, 8 consecutive lanes
// of a wavefront); lane `sub` takes the directions d = sub, sub + LPS, ...  and
// the partial sums are combined with cross-lane shuffles.  R right-hand sides
// that share the gauge field are processed together so that each link entry is
// loaded once for all of them.
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

template <int LPS, typename T> __device__ __forceinline__ T lane_sum(T v)
{
#pragma unroll
    for (int o = LPS / 2; o >= 1; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// acc[r][a] += sum over this lane's directions of L_d(s)[a][b] in_r(n_d(s))[b]
template <class P, int LPS, int R>
__device__ __forceinline__ void hop_accumulate(const Geom &g, const typename P::link_t *__restrict__ links,
                                               const int32_t *__restrict__ nbr, int p_out, int s, int sub,
                                               const void *const *in, const bool *act,
                                               cplx<typename P::real> (*acc)[3])
{
    using real = typename P::real;
    SiteCoord c;
    if (!nbr)
        c = decode_site(g, p_out, s);
#pragma unroll
    for (int j = 0; j < 8 / LPS; ++j) {
        const int d = sub + j * LPS;
        const int n = nbr ? nbr[(int64_t)d * g.Vh + s] : neighbour(g, c, s, d);
        cplx<real> U[9];
        const typename P::link_t *lp = links + (int64_t)d * 9 * g.Vh + s;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            U[k] = P::load_link(lp + (int64_t)k * g.Vh);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!act[r])
                continue;
            cplx<real> chi[3];
            P::load_spinor(in[r], g.Vh, n, chi);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    cmac(acc[r][a], U[a * 3 + b], chi[b]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc[r][a].re = lane_sum<LPS>(acc[r][a].re);
            acc[r][a].im = lane_sum<LPS>(acc[r][a].im);
        }
}

// Colour c of an output site is written / reduced by lane (c mod LPS).
template <int LPS> __device__ __forceinline__ bool owns_colour(int sub, int c) { return (c % LPS) == sub; }

// ---- block reductions (deterministic: fixed shuffle tree, fixed LDS order) ----

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
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

// Per-block partial sums are published with a device-scope store followed by a
// device-scope fence by the writing thread; the block then takes a ticket from
// a device-scope atomic counter.  The block that draws the last ticket fences
// again before reading the partials, so it sees every block's value even when
// the blocks ran on different XCDs (each XCD has its own L2).
__device__ __forceinline__ void publish_partial(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
}

__device__ __forceinline__ bool arrive_last(unsigned *counter, unsigned nblocks, int *lds_flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(counter, 1u);
        const int last = (t == nblocks - 1);
        if (last) {
            __threadfence();
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        *lds_flag = last;
    }
    __syncthreads();
    return *lds_flag != 0;
}

__device__ __forceinline__ double load_partial(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// In the last block: total of partials[0 .. n) in a fixed order; valid in thread 0.
__device__ __forceinline__ double reduce_partials(const double *partials, int n, double *lds)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        v += load_partial(partials + i);
    double arr[1] = {v};
    double out;
    block_sum_multi<1>(arr, lds, out);
    return out;
}

}  // namespace stag
