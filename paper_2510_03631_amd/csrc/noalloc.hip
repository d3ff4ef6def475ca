// Batched Answer for callers that cannot allocate device memory: the
// workspace of pir_answer_batch (limb planes, column sums, split-K
// partials) lives in a fixed array of device memory that the library holds
// on every device it runs on until the process ends.
#include <mutex>

#include "qpir_internal.h"

// The scratch array.  In host code its name is only a stand-in for the
// device copy: kernels and copies get the address resolved per device by
// hipGetSymbolAddress below, never the name.
static __device__ __align__(256) uint8_t scratch[PIR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

std::once_flag g_once[kMaxDevices];
void* g_scratch[kMaxDevices];          // device address of `scratch`, per device
pir_status g_status[kMaxDevices];      // outcome of the lookup, per device

}  // namespace

// Resolve the scratch array's address on `dev`, once; `dev` must be current.
pir_status noalloc_init_device(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return PIR_ERR_UNSUPPORTED;
    std::call_once(g_once[dev], [dev] {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p != nullptr &&
            (uintptr_t)p % kWsAlign == 0) {
            g_scratch[dev] = p;
            g_status[dev] = PIR_OK;
        } else {
            (void)hipGetLastError();
            g_status[dev] = PIR_ERR_DEVICE;
        }
    });
    return g_status[dev];
}

extern "C" pir_status pir_answer_batch_noalloc(pir_db_t* db, const uint32_t* d_Q, uint32_t B,
                                               uint32_t* d_out, pir_stream_t stream) {
    if (!db_ok(db)) return PIR_ERR_INVALID_ARG;
    if (B == 0) return PIR_OK;
    int dev = -1;
    if (!d_Q || !d_out || hipGetDevice(&dev) != hipSuccess || dev != db->device)
        return PIR_ERR_INVALID_ARG;
    if (B > kMaxBatch) return PIR_ERR_SHAPE;
    // Opening the handle resolved the address on this device; this only
    // reads the outcome.
    const pir_status init = noalloc_init_device(dev);
    if (init != PIR_OK) return init;
    BatchPlan plan;
    const pir_status st = mfma_plan_batch(db, B, nullptr, 0, 0, false, &plan);
    if (st != PIR_OK) return st;
    if (plan.need > (size_t)PIR_NOALLOC_SCRATCH_BYTES) return PIR_ERR_SHAPE;
    const BatchIO io{d_Q, B, 1, d_out, B, 1};
    return mfma_run_batch(db, io, B, nullptr, 0, plan, g_scratch[dev], nullptr,
                          static_cast<hipStream_t>(stream));
}
