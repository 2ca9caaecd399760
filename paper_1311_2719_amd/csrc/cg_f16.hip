// CG step kernels, initialisation and tuning probe for the F16 working
// precision, all three link rows stored.
#include "cg_launch.hpp"

namespace stag {

const CgLaunchTable &cg_table_f16() { return TileTable<PrecF16, 3, 1, 2, 3, 4, 6, 8, 12>::table(); }

}  // namespace stag
