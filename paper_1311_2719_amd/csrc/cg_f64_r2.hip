// CG step kernels, initialisation and tuning probe for the F64 working
// precision, two link rows stored, the third rebuilt.
#include "cg_launch.hpp"

namespace stag {

const CgLaunchTable &cg_table_f64_r2() { return TileTable<PrecF64, 2, 1, 2, 4>::table(); }

}  // namespace stag
