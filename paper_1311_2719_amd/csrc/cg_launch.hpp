// Launch tables for the CG / hop kernels of one working precision.  Each
// precision's kernels are instantiated in their own translation unit
// (cg_f64.hip, cg_f32.hip, cg_f16.hip) and reached through cg_table(prec).
#pragma once

#include "cg_kernels.hpp"

namespace stag {

struct CgLaunchTable {
    // K1 / K2 / probe take (lanes per site, right-hand sides per tile)
    hipError_t (*ap)(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a);
    hipError_t (*update)(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a);
    hipError_t (*init)(dim3 grid, dim3 block, hipStream_t s, const CgArgs &a);
    hipError_t (*ru_residual)(int lps, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a);
    // out_r = D in_r over grid.y tiles of R right-hand sides (tiles alternate parity)
    hipError_t (*probe)(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const Geom &g, const void *links,
                        const int32_t *nbr, const void *in, void *out, int remap);
    const int *rtiles;  // right-hand-side tile sizes compiled for this precision
    int n_rtiles;
};

const CgLaunchTable &cg_table(int prec);
hipError_t launch_ru_dx(int lps, bool mixed, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a);

// The table entries for one precision, generated from the kernel templates.
#define STAG_LPS_SWITCH(KERNEL, P, R, ...)                                                     \
    switch (lps) {                                                                          \
    case 1: hipLaunchKernelGGL((KERNEL<P, 1, R>), grid, block, 0, s, __VA_ARGS__); break;   \
    case 2: hipLaunchKernelGGL((KERNEL<P, 2, R>), grid, block, 0, s, __VA_ARGS__); break;   \
    case 4: hipLaunchKernelGGL((KERNEL<P, 4, R>), grid, block, 0, s, __VA_ARGS__); break;   \
    case 8: hipLaunchKernelGGL((KERNEL<P, 8, R>), grid, block, 0, s, __VA_ARGS__); break;   \
    default: return hipErrorInvalidValue;                                                   \
    }

template <class P, int R> struct RLaunch {
    static hipError_t ap(int lps, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a)
    {
        STAG_LPS_SWITCH(k_cg_ap, P, R, a);
        return hipGetLastError();
    }
    static hipError_t update(int lps, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a)
    {
        STAG_LPS_SWITCH(k_cg_update, P, R, a);
        return hipGetLastError();
    }
    static hipError_t probe(int lps, dim3 grid, dim3 block, hipStream_t s, const Geom &g, const void *links,
                            const int32_t *nbr, const void *in, void *out, int remap)
    {
        STAG_LPS_SWITCH(k_hop_probe, P, R, g, links, nbr, in, out, remap);
        return hipGetLastError();
    }
};

template <class P> struct PLaunch {
    static hipError_t init(dim3 grid, dim3 block, hipStream_t s, const CgArgs &a)
    {
        hipLaunchKernelGGL((k_cg_init<P>), grid, block, 0, s, a);
        return hipGetLastError();
    }
    static hipError_t ru_residual(int lps, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a)
    {
        switch (lps) {
        case 1: hipLaunchKernelGGL((k_ru_residual<P, 1>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_ru_residual<P, 2>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_ru_residual<P, 4>), grid, block, 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_ru_residual<P, 8>), grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
};

}  // namespace stag
