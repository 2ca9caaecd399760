// Kernel instantiations and launch table for the F64 working precision.
#include "cg_launch.hpp"

namespace stag {

namespace {

using P = PrecF64;
const int kTiles[] = {1, 2, 4};

hipError_t step1(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int ver)
{
    switch (R) {
    case 1: return RLaunch<P, 1>::step1(lps, grid, block, s, a, ver);
    case 2: return RLaunch<P, 2>::step1(lps, grid, block, s, a, ver);
    case 4: return RLaunch<P, 4>::step1(lps, grid, block, s, a, ver);
    default: return hipErrorInvalidValue;
    }
}

hipError_t step2(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a, int ver)
{
    switch (R) {
    case 1: return RLaunch<P, 1>::step2(lps, grid, block, s, a, ver);
    case 2: return RLaunch<P, 2>::step2(lps, grid, block, s, a, ver);
    case 4: return RLaunch<P, 4>::step2(lps, grid, block, s, a, ver);
    default: return hipErrorInvalidValue;
    }
}

hipError_t probe(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const Geom &g, const void *links,
                 const int32_t *nbr, const void *in, void *out, int remap)
{
    switch (R) {
    case 1: return RLaunch<P, 1>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    case 2: return RLaunch<P, 2>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    case 4: return RLaunch<P, 4>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

const CgLaunchTable &cg_table_f64()
{
    static const CgLaunchTable t = {step1, step2, PLaunch<P>::init,
                                    probe, kTiles, (int)(sizeof(kTiles) / sizeof(kTiles[0]))};
    return t;
}

}  // namespace stag
