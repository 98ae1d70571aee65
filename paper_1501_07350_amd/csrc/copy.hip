// copy.hip -- the copy of one axis pass's access pattern, the measured
// ceiling a pass is compared with besides the HBM peak.
//
// A pass of the plan moves each element of the grid from HBM and back once,
// in tiles of W lines: strided lines are read and written with the lanes of
// a wavefront walking W consecutive columns of a row, contiguous lines with
// the lanes walking along the line (or as one flat block through LDS when a
// line has fewer than kDirectRowMinTpl threads).  The copy here launches the
// same tiles (same W, same W * TPL threads, same tile order and grid-data
// access mode) and has every thread load the elements of its first-stage
// butterflies -- positions b + r * L/R0 of its line, b = t + i * TPL -- in one
// burst, as the pass does, then store them to the same positions of `out`.
// No arithmetic and no LDS exchange, so its time is what the pass's memory
// accesses alone cost on this device.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/offt.h"
#include "offt_internal.h"
#include "plan_impl.h"

namespace offt {

struct CopyArgs {
    const void* in;
    void* out;
    int64_t nlines, M2;
    int L, logW, tpl, r0, nb;   // line length, log2 lines per tile, threads per line, first radix, butterflies per thread
    int mode;                   // 0 contiguous lines, 1 strided lines
    int flat;                   // contiguous lines staged as one flat block (threads per line < kDirectRowMinTpl)
    int xcd_remap;
    int stream_io;
};

template <typename V, int KMAX, int MAXT>
__global__ void __launch_bounds__(MAXT) copy_pattern_kernel(CopyArgs a) {
    const V* __restrict__ in = static_cast<const V*>(a.in);
    V* __restrict__ out = static_cast<V*>(a.out);
    const int W = 1 << a.logW;
    const int tid = threadIdx.x;
    const int64_t l0 = xcd_tile(blockIdx.x, gridDim.x, a.xcd_remap) << a.logW;
    const int64_t rem = a.nlines - l0;
    const int nl = rem < W ? (int)rem : W;
    const bool nt = a.stream_io != 0;
    if (a.mode == 0 && a.flat) {
        const int NT = W * a.tpl;
        const int64_t base = l0 * a.L;
        for (int f = tid; f < nl * a.L; f += NT) store_io(out + base + f, load_io(in + base + f, nt), nt);
        return;
    }
    int w, t;
    if (a.mode == 1) {
        w = tid & (W - 1);
        t = tid >> a.logW;
    } else {
        w = tid / a.tpl;
        t = tid % a.tpl;
    }
    if (w >= nl) return;
    const int64_t l = l0 + w;
    int64_t base, stride;
    if (a.mode == 1) {
        const int64_t m1 = l / a.M2, m2 = l - m1 * a.M2;
        base = m1 * (int64_t)a.L * a.M2 + m2;
        stride = a.M2;
    } else {
        base = l * a.L;
        stride = 1;
    }
    const int B = a.L / a.r0;   // butterflies of the first stage
    V v[KMAX];
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        const int i = s % a.nb, r = s / a.nb;   // register slot s = r * nb + i
        const int b = t + i * a.tpl;
        if (r < a.r0 && b < B) v[s] = load_io(in + base + (int64_t)(b + r * B) * stride, nt);
    }
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        const int i = s % a.nb, r = s / a.nb;
        const int b = t + i * a.tpl;
        if (r < a.r0 && b < B) store_io(out + base + (int64_t)(b + r * B) * stride, v[s], nt);
    }
}

template <typename V, int KMAX, int MAXT>
static hipError_t launch_copy(const CopyArgs& a, int64_t nblocks, int threads, hipStream_t s) {
    hipLaunchKernelGGL((copy_pattern_kernel<V, KMAX, MAXT>), dim3((unsigned)nblocks), dim3(threads), 0, s, a);
    return hipGetLastError();
}

}  // namespace offt

using namespace offt;

extern "C" {

int offt_copy_pass(offt_plan_t p, int i, const void* in, void* out, void* stream) {
    if (!p || !in || !out || in == out) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    if (p->kind != 1 && p->kind != 3) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    if (i < 0 || i >= p->npass) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    const PassPlan& pp = dir_passes(p, OFFT_FORWARD)[i];
    if (pp.mode >= 2) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }   // transposing passes
    CopyArgs a;
    a.in = in;
    a.out = out;
    a.nlines = pp.M1 * pp.M2;
    a.M2 = pp.M2;
    a.L = pp.L;
    a.logW = pp.logW;
    a.tpl = pp.k->tpl;
    a.r0 = pp.k->radices[0];
    a.nb = (pp.L / a.r0 + a.tpl - 1) / a.tpl;
    a.mode = pp.mode;
    a.flat = pp.mode == 0 && a.tpl < kDirectRowMinTpl;
    a.xcd_remap = pp.xcd;
    a.stream_io = pp.stream;
    const int64_t W = int64_t(1) << pp.logW;
    const int64_t nblocks = (a.nlines + W - 1) / W;
    const int threads = (int)(W * a.tpl);
    const int k = a.nb * a.r0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (p->dtype == OFFT_C2C_F64) {
        if (threads > 512) e = hipErrorInvalidValue;
        else if (k <= 8) e = launch_copy<double2, 8, 512>(a, nblocks, threads, s);
        else if (k <= 16) e = launch_copy<double2, 16, 512>(a, nblocks, threads, s);
        else if (k <= 32) e = launch_copy<double2, 32, 512>(a, nblocks, threads, s);
        else e = hipErrorInvalidValue;
    } else {
        if (k <= 8) e = launch_copy<float2, 8, 1024>(a, nblocks, threads, s);
        else if (k <= 16) e = launch_copy<float2, 16, 1024>(a, nblocks, threads, s);
        else if (k <= 32) e = launch_copy<float2, 32, 1024>(a, nblocks, threads, s);
        else if (k <= 64 && threads <= 512) e = launch_copy<float2, 64, 512>(a, nblocks, threads, s);
        else e = hipErrorInvalidValue;
    }
    const int rc = e == hipSuccess ? OFFT_SUCCESS : (e == hipErrorInvalidValue ? OFFT_ERR_UNSUPPORTED_SIZE : OFFT_ERR_HIP);
    set_error(rc);
    return rc;
}

}  // extern "C"
