// sweep_d2.hip -- line-solve kernels for double state, degree 2.
#include "sweep_kernels.h"

namespace iga {
SweepFn pick_sweep_d2(int mm, bool diry) { return pick_mm<double, 2>(mm, diry); }
SweepBatchFn pick_sweep_batch_d2(int mm, bool diry) { return pick_mm_batch<double, 2>(mm, diry); }

}  // namespace iga
