// noalloc.hip -- the 3-D transform for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc): the heuristic plan of offt_plan without a plan object, its
// twiddle tables written into a file-scope device array instead of
// plan-owned allocations.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/offt.h"
#include "offt_internal.h"
#include "plan_impl.h"

namespace offt {

// One twiddle table per distinct axis length, up to OFFT_MAX_AXIS complex
// binary64 values each.
constexpr size_t kScratchTableBytes = (size_t)OFFT_MAX_AXIS * 16;
constexpr size_t kScratchBytes = 3 * kScratchTableBytes;   // 48 KiB

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device, looked up once per device with that
// device current (the array's host-side name is not a device address).
constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mutex;

static int scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return OFFT_ERR_NO_DEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) return OFFT_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return OFFT_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return OFFT_SUCCESS;
}

}  // namespace offt

using namespace offt;

extern "C" {

int offt_exec_noalloc(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch, int direction, int normalize,
                      const void* in, void* out, void* stream) {
    int rc = validate_dims(Na, Nb, Nc, dtype, batch);
    if (rc == OFFT_SUCCESS && (!in || !out || (direction != OFFT_FORWARD && direction != OFFT_BACKWARD) ||
                               (normalize != 0 && normalize != 1)))
        rc = OFFT_ERR_INVALID_ARG;
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    void* base = nullptr;
    rc = check_device();
    if (rc == OFFT_SUCCESS) rc = scratch_address(&base);
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t dims[3] = {Na, Nb, Nc};
    // the heuristic plan of offt_plan (host-side choice, nothing allocated)
    PassPlan passes[3];
    const int npass = build_passes(default_choice(dtype, dims), dims, batch, passes);
    for (int i = 0; i < npass; ++i)
        if (!passes[i].k) { set_error(OFFT_ERR_UNSUPPORTED_SIZE); return OFFT_ERR_UNSUPPORTED_SIZE; }
    // one table per distinct length in the scratch array, written before the
    // passes on the same stream (every call rewrites them)
    int lens[3] = {0, 0, 0};
    int nlen = 0;
    for (int i = 0; i < npass; ++i) {
        int slot = 0;
        while (slot < nlen && lens[slot] != passes[i].L) ++slot;
        if (slot == nlen) {
            if ((size_t)passes[i].L * elem_size(dtype) > kScratchTableBytes) {
                set_error(OFFT_ERR_UNSUPPORTED_SIZE);
                return OFFT_ERR_UNSUPPORTED_SIZE;
            }
            lens[nlen++] = passes[i].L;
            void* tw = static_cast<char*>(base) + (size_t)slot * kScratchTableBytes;
            if (launch_twiddles(tw, passes[i].L, dtype, s) != hipSuccess) {
                (void)hipGetLastError();
                set_error(OFFT_ERR_HIP);
                return OFFT_ERR_HIP;
            }
        }
        passes[i].tw = static_cast<char*>(base) + (size_t)slot * kScratchTableBytes;
    }
    // the passes, as offt_exec_fwd / offt_exec_bwd run them (a plan object on
    // the stack only carries the shape and the scaling)
    offt_plan_s view;
    view.kind = 1;
    view.dtype = dtype;
    view.dims[0] = Na; view.dims[1] = Nb; view.dims[2] = Nc;
    view.batch = batch;
    view.normalize = normalize;
    rc = exec_passes(&view, passes, npass, in, out, nullptr, direction, s);
    set_error(rc);
    return rc;
}

}  // extern "C"
