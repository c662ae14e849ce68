// sweep_d3.hip -- line-solve kernels for double state, degree 3.
#include "sweep_kernels.h"

namespace iga {
SweepFn pick_sweep_d3(int lw, int mm, bool diry) { return pick_lw_mm<double, 3>(lw, mm, diry); }
}  // namespace iga
