// sweep_f2.hip -- line-solve kernels for float state, degree 2.
#include "sweep_win.h"

namespace iga {
SweepFn pick_sweep_f2(int mm, bool diry) { return pick_mm<float, 2>(mm, diry); }
SweepBatchFn pick_sweep_batch_f2(int mm, bool diry) { return pick_mm_batch<float, 2>(mm, diry); }

WSweepFn pick_wsweep_f2(int mm, bool diry, bool one) { return pick_wmm<float, 2>(mm, diry, one); }
WSweepBatchFn pick_wsweep_batch_f2(int mm, bool diry, bool one) {
    return pick_wmm_batch<float, 2>(mm, diry, one);
}

}  // namespace iga
