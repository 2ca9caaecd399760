// CG step kernels, initialisation, tuning probe and shared-link tiles for the F32 working
// precision, two link rows stored, the third rebuilt.
#include "cg_launch.hpp"

namespace stag {

const CgLaunchTable &cg_table_f32_r2()
{
    return with_shared<TileTable<PrecF32, 2, 1, 2, 3, 4, 6, 8, 12>, SharedTable<PrecF32, 2, STAG_SHARED_SHAPES>>();
}

}  // namespace stag
