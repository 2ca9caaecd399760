// CG step kernels, initialisation and tuning probe for the F64 working
// precision with non-temporal link loads (fields beyond the Infinity Cache),
// two link rows stored, the third rebuilt.
#include "cg_launch.hpp"

namespace stag {

const CgLaunchTable &cg_table_f64nt_r2() { return TileTable<PrecF64NT, 2, 1, 2, 4>::table(); }

}  // namespace stag
