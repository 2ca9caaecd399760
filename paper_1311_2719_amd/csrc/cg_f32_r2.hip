// CG step kernels, initialisation and tuning probe for the F32 working
// precision, two link rows stored, the third rebuilt.
#include "cg_launch.hpp"

namespace stag {

const CgLaunchTable &cg_table_f32_r2() { return TileTable<PrecF32, 2, 1, 2, 3, 4, 6, 8, 12>::table(); }

}  // namespace stag
