// Launch tables for the CG / hop kernels of one working precision and link
// format.  Each (precision, link rows) pair is instantiated in its own
// translation unit (cg_f64.hip, cg_f64_r2.hip, ...) and reached through
// cg_table(prec, rows, nt_links).
#pragma once

#include "cg_shared.hpp"

namespace stag {

struct CgLaunchTable {
    // K1 / K2 / probe take (lanes per site, right-hand sides per tile); ver
    // selects the state and partial-sum buffers the step reads
    hipError_t (*step1)(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int ver);
    hipError_t (*step2)(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int ver);
    hipError_t (*init)(dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int lps);
    // out_r = D in_r over grid.y tiles of R right-hand sides (tiles alternate parity)
    hipError_t (*probe)(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const Geom &g, const void *links,
                        const int32_t *nbr, const void *in, void *out, int remap);
    const int *rtiles;  // right-hand-side tile sizes compiled for this precision
    int n_rtiles;
    // shared-link tiles (FP32 / FP16 working precision; null otherwise): W
    // wavefronts per block, R / W systems each, the block's links staged in
    // LDS; stiles lists the compiled shapes as shared_code(W, R / W)
    hipError_t (*shared1)(int R, int W, dim3 grid, hipStream_t s, const CgArgs &a, int ver);
    hipError_t (*shared2)(int R, int W, dim3 grid, hipStream_t s, const CgArgs &a, int ver);
    const int *stiles;
    int n_stiles;
};

const CgLaunchTable &cg_table(int prec, int rows, int nt_links);

// One kernel of the table for every lanes-per-site value.
#define STAG_LPS_SWITCH(KERNEL, P, R, ROWS, ...)                                                    \
    switch (lps) {                                                                                 \
    case 1: hipLaunchKernelGGL((KERNEL<P, 1, R, ROWS>), grid, block, 0, s, __VA_ARGS__); break;    \
    case 2: hipLaunchKernelGGL((KERNEL<P, 2, R, ROWS>), grid, block, 0, s, __VA_ARGS__); break;    \
    case 4: hipLaunchKernelGGL((KERNEL<P, 4, R, ROWS>), grid, block, 0, s, __VA_ARGS__); break;    \
    case 8: hipLaunchKernelGGL((KERNEL<P, 8, R, ROWS>), grid, block, 0, s, __VA_ARGS__); break;    \
    default: return hipErrorInvalidValue;                                                          \
    }

template <class P, int R, int ROWS> struct RLaunch {
    static hipError_t step1(int lps, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int ver)
    {
        STAG_LPS_SWITCH(k_cg_step1, P, R, ROWS, a, ver);
        return hipGetLastError();
    }
    static hipError_t step2(int lps, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int ver)
    {
        STAG_LPS_SWITCH(k_cg_step2, P, R, ROWS, a, ver);
        return hipGetLastError();
    }
    static hipError_t probe(int lps, dim3 grid, dim3 block, hipStream_t s, const Geom &g, const void *links,
                            const int32_t *nbr, const void *in, void *out, int remap)
    {
        STAG_LPS_SWITCH(k_hop_probe, P, R, ROWS, g, links, nbr, in, out, remap);
        return hipGetLastError();
    }
};

template <class P> struct PLaunch {
    static hipError_t init(dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int lps)
    {
        hipLaunchKernelGGL((k_cg_init<P>), grid, block, 0, s, a, lps);
        return hipGetLastError();
    }
};

// The table of precision P, link rows ROWS and right-hand-side tiles Rs...:
// a tile size not in Rs is rejected with hipErrorInvalidValue.
template <class P, int ROWS, int... Rs> struct TileTable {
    static constexpr int tiles[] = {Rs...};

    static hipError_t step1(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int ver)
    {
        hipError_t e = hipErrorInvalidValue;
        (void)((R == Rs && ((e = RLaunch<P, Rs, ROWS>::step1(lps, grid, block, s, a, ver)), true)) || ...);
        return e;
    }
    static hipError_t step2(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int ver)
    {
        hipError_t e = hipErrorInvalidValue;
        (void)((R == Rs && ((e = RLaunch<P, Rs, ROWS>::step2(lps, grid, block, s, a, ver)), true)) || ...);
        return e;
    }
    static hipError_t probe(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const Geom &g, const void *links,
                            const int32_t *nbr, const void *in, void *out, int remap)
    {
        hipError_t e = hipErrorInvalidValue;
        (void)((R == Rs && ((e = RLaunch<P, Rs, ROWS>::probe(lps, grid, block, s, g, links, nbr, in, out, remap)),
                            true)) ||
               ...);
        return e;
    }
    static const CgLaunchTable &table()
    {
        static const CgLaunchTable t = {step1, step2, PLaunch<P>::init, probe, tiles, (int)sizeof...(Rs),
                                        nullptr, nullptr, nullptr, 0};
        return t;
    }
};

template <class P, int W, int RR, int ROWS> struct SLaunch {
    static hipError_t step1(dim3 grid, hipStream_t s, const CgArgs &a, int ver)
    {
        hipLaunchKernelGGL((k_cg_shared1<P, W, RR, ROWS>), grid, dim3(64 * W), 0, s, a, ver);
        return hipGetLastError();
    }
    static hipError_t step2(dim3 grid, hipStream_t s, const CgArgs &a, int ver)
    {
        hipLaunchKernelGGL((k_cg_shared2<P, W, RR, ROWS>), grid, dim3(64 * W), 0, s, a, ver);
        return hipGetLastError();
    }
};

// Shape code of a shared-link tile: RR systems per wavefront, W wavefronts
// per block (tile R = W RR, block = 64 W threads).
constexpr int shared_code(int W, int RR) { return RR * 100 + W; }

// The shared-link kernels of precision P and link rows ROWS for the shapes
// Codes... (shared_code values); a shape not in the list is rejected.
template <class P, int ROWS, int... Codes> struct SharedTable {
    static constexpr int tiles[] = {Codes...};

    static hipError_t shared1(int R, int W, dim3 grid, hipStream_t s, const CgArgs &a, int ver)
    {
        hipError_t e = hipErrorInvalidValue;
        (void)(((W > 0 && R % W == 0 && shared_code(W, R / W) == Codes) &&
                ((e = SLaunch<P, Codes % 100, Codes / 100, ROWS>::step1(grid, s, a, ver)), true)) ||
               ...);
        return e;
    }
    static hipError_t shared2(int R, int W, dim3 grid, hipStream_t s, const CgArgs &a, int ver)
    {
        hipError_t e = hipErrorInvalidValue;
        (void)(((W > 0 && R % W == 0 && shared_code(W, R / W) == Codes) &&
                ((e = SLaunch<P, Codes % 100, Codes / 100, ROWS>::step2(grid, s, a, ver)), true)) ||
               ...);
        return e;
    }
};

// The shapes compiled for FP32 and FP16: one system per wavefront for tiles
// of 2 to 16, two for tiles of 4 to 16, three for tiles of 3, 6 and 12.
#define STAG_SHARED_SHAPES                                                                                   \
    shared_code(2, 1), shared_code(3, 1), shared_code(4, 1), shared_code(6, 1), shared_code(8, 1),            \
        shared_code(12, 1), shared_code(16, 1), shared_code(2, 2), shared_code(3, 2), shared_code(4, 2),      \
        shared_code(6, 2), shared_code(8, 2), shared_code(1, 3), shared_code(2, 3), shared_code(4, 3)

// A register-tile table with the shared-link kernels of S added.
template <class T, class S> const CgLaunchTable &with_shared()
{
    static const CgLaunchTable t = [] {
        CgLaunchTable x = T::table();
        x.shared1 = S::shared1;
        x.shared2 = S::shared2;
        x.stiles = S::tiles;
        x.n_stiles = (int)(sizeof(S::tiles) / sizeof(S::tiles[0]));
        return x;
    }();
    return t;
}

}  // namespace stag
