// sweep_d2.hip -- line-solve kernels for double state, degree 2.
#include "sweep_kernels.h"

namespace iga {
SweepFn pick_sweep_d2(int lw, int mm, bool diry) { return pick_lw_mm<double, 2>(lw, mm, diry); }
}  // namespace iga
