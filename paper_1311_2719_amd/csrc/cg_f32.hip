// Kernel instantiations and launch table for the F32 working precision.
#include "cg_launch.hpp"

namespace stag {

namespace {

using P = PrecF32;
const int kTiles[] = {1, 2, 3, 4, 6, 8, 12};

hipError_t ap(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a)
{
    switch (R) {
    case 1: return RLaunch<P, 1>::ap(lps, grid, block, s, a);
    case 2: return RLaunch<P, 2>::ap(lps, grid, block, s, a);
    case 3: return RLaunch<P, 3>::ap(lps, grid, block, s, a);
    case 4: return RLaunch<P, 4>::ap(lps, grid, block, s, a);
    case 6: return RLaunch<P, 6>::ap(lps, grid, block, s, a);
    case 8: return RLaunch<P, 8>::ap(lps, grid, block, s, a);
    case 12: return RLaunch<P, 12>::ap(lps, grid, block, s, a);
    default: return hipErrorInvalidValue;
    }
}

hipError_t update(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const CgArgs &a)
{
    switch (R) {
    case 1: return RLaunch<P, 1>::update(lps, grid, block, s, a);
    case 2: return RLaunch<P, 2>::update(lps, grid, block, s, a);
    case 3: return RLaunch<P, 3>::update(lps, grid, block, s, a);
    case 4: return RLaunch<P, 4>::update(lps, grid, block, s, a);
    case 6: return RLaunch<P, 6>::update(lps, grid, block, s, a);
    case 8: return RLaunch<P, 8>::update(lps, grid, block, s, a);
    case 12: return RLaunch<P, 12>::update(lps, grid, block, s, a);
    default: return hipErrorInvalidValue;
    }
}

hipError_t probe(int lps, int R, dim3 grid, dim3 block, hipStream_t s, const Geom &g, const void *links,
                 const int32_t *nbr, const void *in, void *out, int remap)
{
    switch (R) {
    case 1: return RLaunch<P, 1>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    case 2: return RLaunch<P, 2>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    case 3: return RLaunch<P, 3>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    case 4: return RLaunch<P, 4>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    case 6: return RLaunch<P, 6>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    case 8: return RLaunch<P, 8>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    case 12: return RLaunch<P, 12>::probe(lps, grid, block, s, g, links, nbr, in, out, remap);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

const CgLaunchTable &cg_table_f32()
{
    static const CgLaunchTable t = {ap, update, PLaunch<P>::init, PLaunch<P>::ru_residual,
                                    probe, kTiles, (int)(sizeof(kTiles) / sizeof(kTiles[0]))};
    return t;
}

}  // namespace stag
