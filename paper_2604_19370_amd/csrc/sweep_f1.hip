// sweep_f1.hip -- line-solve kernels for float state, degree 1.
#include "sweep_win.h"

namespace iga {
SweepFn pick_sweep_f1(int mm, bool diry) { return pick_mm<float, 1>(mm, diry); }
SweepBatchFn pick_sweep_batch_f1(int mm, bool diry) { return pick_mm_batch<float, 1>(mm, diry); }

WSweepFn pick_wsweep_f1(int mm, bool diry, bool one) { return pick_wmm<float, 1>(mm, diry, one); }
WSweepBatchFn pick_wsweep_batch_f1(int mm, bool diry, bool one) {
    return pick_wmm_batch<float, 1>(mm, diry, one);
}

}  // namespace iga
