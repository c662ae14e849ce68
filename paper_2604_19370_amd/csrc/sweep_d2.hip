// sweep_d2.hip -- line-solve kernels for double state, degree 2.
#include "sweep_win.h"

namespace iga {
SweepFn pick_sweep_d2(int mm, bool diry) { return pick_mm<double, 2>(mm, diry); }
SweepBatchFn pick_sweep_batch_d2(int mm, bool diry) { return pick_mm_batch<double, 2>(mm, diry); }

WSweepFn pick_wsweep_d2(int mm, bool diry, bool one) { return pick_wmm<double, 2>(mm, diry, one); }
WSweepBatchFn pick_wsweep_batch_d2(int mm, bool diry, bool one) {
    return pick_wmm_batch<double, 2>(mm, diry, one);
}

}  // namespace iga
