// CG step kernels, initialisation, tuning probe and shared-link tiles for the F16 working
// precision, all three link rows stored.
#include "cg_launch.hpp"

namespace stag {

const CgLaunchTable &cg_table_f16()
{
    return with_shared<TileTable<PrecF16, 3, 1, 2, 3, 4, 6, 8, 12>, SharedTable<PrecF16, 3, STAG_SHARED_SHAPES>>();
}

}  // namespace stag
