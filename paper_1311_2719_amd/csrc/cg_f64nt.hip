// CG step kernels, initialisation and tuning probe for the F64 working
// precision with non-temporal link loads (fields beyond the Infinity Cache),
// all three link rows stored.
#include "cg_launch.hpp"

namespace stag {

const CgLaunchTable &cg_table_f64nt() { return TileTable<PrecF64NT, 3, 1, 2, 4>::table(); }

}  // namespace stag
