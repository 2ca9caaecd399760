// CG step kernels, initialisation and tuning probe for the F32 working
// precision, all three link rows stored.
#include "cg_launch.hpp"

namespace stag {

const CgLaunchTable &cg_table_f32() { return TileTable<PrecF32, 3, 1, 2, 3, 4, 6, 8, 12>::table(); }

}  // namespace stag
