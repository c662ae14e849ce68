// sweep_d1.hip -- line-solve kernels for double state, degree 1.
#include "sweep_win.h"

namespace iga {
SweepFn pick_sweep_d1(int mm, bool diry) { return pick_mm<double, 1>(mm, diry); }
SweepBatchFn pick_sweep_batch_d1(int mm, bool diry) { return pick_mm_batch<double, 1>(mm, diry); }

WSweepFn pick_wsweep_d1(int mm, bool diry, bool one) { return pick_wmm<double, 1>(mm, diry, one); }
WSweepBatchFn pick_wsweep_batch_d1(int mm, bool diry, bool one) {
    return pick_wmm_batch<double, 1>(mm, diry, one);
}

}  // namespace iga
