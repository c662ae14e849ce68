// noalloc.cpp -- iga_step_noalloc: one time step whose right-hand-side
// scratch lives in a file-scope device array instead of the plan's own
// buffers, for callers that cannot allocate device memory.
//
// The array `scratch` is a device symbol: in host code its name is only a
// stand-in, so its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels.  Each GPU holds its own copy of the array, which keeps
// the contents of the last call on that GPU.  The step overwrites every
// right-hand-side entry before it reads it, so nothing has to be cleared.
#include <mutex>

#include "iga_internal.h"

namespace {

// Right-hand sides of one step: 2 fields (4 under column-wave x sweeps).
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;   // IGA_NOALLOC_SCRATCH_BYTES
static_assert(SCRATCH_BYTES == IGA_NOALLOC_SCRATCH_BYTES, "header and source disagree");

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_lock;
void *g_ptr[MAX_DEVICES] = {};   // device address of `scratch`, per device ordinal

iga_status scratch_address(void **out)
{
    int dev = -1;
    IGA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return iga::fail(IGA_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        IGA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return iga::fail(IGA_EDEVICE, "hipGetSymbolAddress returned NULL");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return IGA_OK;
}

}  // namespace

using namespace iga;

extern "C" iga_status iga_step_noalloc(iga_plan *plan, void *T, void *fuel, void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    iga_status st;
    if ((st = check_field(T, "T")) || (st = check_field(fuel, "fuel"))) return st;
    if (T == fuel) return fail(IGA_EINVAL, "T and fuel must be different buffers");
    if (!plan->factored) return fail(IGA_ESTATE, "iga_factor_1d has not been called");
    // fields rounded up to 256 bytes so each starts aligned
    const size_t field = (plan->ndof * plan->wsize + 255) & ~size_t(255);
    const int nfields = plan->sched[0].col ? 4 : 2;
    if (nfields * field > SCRATCH_BYTES)
        return fail(IGA_EINVAL, "iga_step_noalloc: the plan needs " +
                                    std::to_string(nfields * field) + " bytes of scratch, above " +
                                    std::to_string(SCRATCH_BYTES));
    void *base = nullptr;
    if ((st = scratch_address(&base))) return st;
    unsigned char *b = static_cast<unsigned char *>(base);
    void *work[4] = {b, b + field, b + 2 * field, b + 3 * field};
    return step_impl(plan, T, fuel, static_cast<hipStream_t>(stream), nullptr, nullptr, work);
}
