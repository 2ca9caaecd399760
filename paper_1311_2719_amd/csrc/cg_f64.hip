// CG step kernels, initialisation and tuning probe for the F64 working
// precision, all three link rows stored.
#include "cg_launch.hpp"

namespace stag {

const CgLaunchTable &cg_table_f64() { return TileTable<PrecF64, 3, 1, 2, 4>::table(); }

}  // namespace stag
