// tuner.cpp -- run-time plan selection at plan time, the GPU counterpart of
// the paper's auto-tuning of communication methods (Sec. 3.2.3): every
// candidate plan is executed a few times during initialization and the
// fastest is kept; a plan cache plays the role of the paper's "User-select
// after tuning once".  Candidates: radix sequence (with the parts its LDS
// exchanges run in) and tile width per axis, and the axis order of the
// passes.
//
// Protocol: 1 warm-up + `reps` timed executions per candidate (hipEvents on the
// tuning stream), score = minimum; ties go to the earlier candidate (the
// heuristic's choices come first).  The data is refilled with uniform random
// values before each candidate (timings on all-zero buffers are not
// representative of real data on this device).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <algorithm>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/offt.h"
#include "offt_internal.h"
#include "plan_impl.h"
#include "selector.h"

namespace offt {

static std::string device_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string n = prop.gcnArchName;
    for (char& ch : n)
        if (ch == ' ' || ch == '\t') ch = '_';
    return n;
}

std::string cache_key(int dtype, const int64_t dims[3], int64_t batch) {
    char buf[256];
    snprintf(buf, sizeof buf, "dtype=%d dims=%lldx%lldx%lld batch=%lld dev=%s", dtype, (long long)dims[0],
             (long long)dims[1], (long long)dims[2], (long long)batch, device_name().c_str());
    return buf;
}

// Returns OFFT_SUCCESS and fills *c when the cache holds a usable entry.
static int cache_lookup(const char* path, int dtype, const int64_t dims[3], int64_t batch, PlanChoice* c) {
    std::ifstream f(path);
    if (!f) return OFFT_ERR_IO;
    const std::string key = cache_key(dtype, dims, batch);
    std::string line;
    int rc = OFFT_ERR_IO;
    while (std::getline(f, line)) {
        const size_t t1 = line.find('\t');
        if (t1 == std::string::npos || line.compare(0, t1, key) != 0 || t1 != key.size()) continue;
        const size_t t2 = line.find('\t', t1 + 1);
        const std::string plan = line.substr(t1 + 1, t2 == std::string::npos ? std::string::npos : t2 - t1 - 1);
        PlanChoice pc;
        if (choice_from_string(plan.c_str(), dtype, dims, &pc)) {
            *c = pc;   // the latest valid entry wins
            rc = OFFT_SUCCESS;
        }
    }
    return rc;
}

static void cache_store(const char* path, int dtype, const int64_t dims[3], int64_t batch,
                        const PlanChoice& c, float ms) {
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    f << cache_key(dtype, dims, batch) << '\t' << choice_to_string(c, dims) << '\t' << ms << '\n';
}

// Times one candidate from `src` to `dst` (equal: in place).  Returns
// OFFT_SUCCESS and the minimum time in *ms.
int time_choice(offt_plan_s* p, const PlanChoice& c, void* src, void* dst, hipStream_t s, int reps, float* ms) {
    PassPlan passes[3];
    const int n = build_passes(c, p->dims, p->batch, passes);
    for (int i = 0; i < n; ++i)
        if (!passes[i].k) return OFFT_ERR_UNSUPPORTED_SIZE;
    int rc = attach_twiddles(p, passes, n, s);
    if (rc != OFFT_SUCCESS) return rc;
    // fresh random data per candidate: unnormalised transforms repeated in
    // place would otherwise grow the values towards overflow
    if (launch_fill_uniform(src, p->dims[0] * p->dims[1] * p->dims[2] * p->batch, p->dtype, 1501, s) != hipSuccess)
        return OFFT_ERR_HIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return OFFT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return OFFT_ERR_HIP; }
    rc = exec_passes(p, passes, n, src, dst, OFFT_FORWARD, s);   // warm-up
    float best = 1e30f;
    for (int r = 0; r < reps && rc == OFFT_SUCCESS; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) { rc = OFFT_ERR_HIP; break; }
        rc = exec_passes(p, passes, n, src, dst, OFFT_FORWARD, s);
        if (rc != OFFT_SUCCESS) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = OFFT_ERR_HIP; break; }
        float t = 0.f;
        if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) { rc = OFFT_ERR_HIP; break; }
        if (t < best) best = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return rc;
}

// Times one axis pass of a plan alone (in place on buf): 1 warm-up + reps runs, minimum.
static int time_pass(offt_plan_s* p, const PlanChoice& c, int axis, void* buf, hipStream_t s, int reps, float* ms) {
    PassPlan passes[3];
    const int n = build_passes(c, p->dims, p->batch, passes);
    int i = 0;
    while (i < n && passes[i].axis != axis) ++i;
    if (i == n || !passes[i].k) return OFFT_ERR_UNSUPPORTED_SIZE;
    int rc = attach_twiddles(p, &passes[i], 1, s);
    if (rc != OFFT_SUCCESS) return rc;
    if (launch_fill_uniform(buf, p->dims[0] * p->dims[1] * p->dims[2] * p->batch, p->dtype, 1502, s) != hipSuccess)
        return OFFT_ERR_HIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return OFFT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return OFFT_ERR_HIP; }
    if (launch_pass(passes[i], buf, buf, 0, 0, 1.0, s) != hipSuccess) rc = OFFT_ERR_HIP;   // warm-up
    float best = 1e30f;
    for (int r = 0; r < reps && rc == OFFT_SUCCESS; ++r) {
        float t = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess || launch_pass(passes[i], buf, buf, 0, 0, 1.0, s) != hipSuccess ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            rc = OFFT_ERR_HIP;
            break;
        }
        best = std::min(best, t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return rc;
}

// Exhaustive search over a factorised space: the passes are independent
// kernels, so every (radix sequence, threads per line, tile width) of each
// axis is timed as a single pass and the fastest kept per axis; then the six
// pass orders are timed as whole transforms with those kernels.  Ties keep
// the earlier candidate (the heuristic's kernels and order come first).
static int exhaustive(offt_plan_s* p, const offt_opts& o, PlanChoice* choice) {
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    const size_t bytes = (size_t)(p->dims[0] * p->dims[1] * p->dims[2] * p->batch) * elem_size(p->dtype);
    // two buffers: whole transforms are timed out of place (src -> buf) unless
    // the caller tunes for in-place use; single passes run in place on buf
    void* buf = nullptr;
    void* src = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) { (void)hipGetLastError(); return OFFT_ERR_OUT_OF_MEMORY; }
    if (o.tune_inplace) {
        src = buf;
    } else if (hipMalloc(&src, bytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(buf);
        return OFFT_ERR_OUT_OF_MEMORY;
    }
    // the timed buffers are filled with random values before every candidate
    int rc = OFFT_SUCCESS;
    PlanChoice best = default_choice(p->dtype, p->dims);
    int timed = 0;
    for (int ax = 0; ax < 3 && rc == OFFT_SUCCESS; ++ax) {
        if (p->dims[ax] <= 1) continue;
        float best_ms = 1e30f;
        PlanChoice cur = best;
        const int lw0 = best.logW[ax];
        // the heuristic's kernel first, so ties keep it
        std::vector<const KernelEntry*> ks = kernels_for(p->dtype, (int)p->dims[ax]);
        std::stable_partition(ks.begin(), ks.end(), [&](const KernelEntry* k) { return k == best.k[ax]; });
        const KernelEntry* best_k = best.k[ax];
        int best_lw = lw0;
        int64_t m2 = 1;
        for (int j = ax + 1; j < 3; ++j) m2 *= p->dims[j];
        for (const KernelEntry* k : ks) {
            // kernels whose LDS exchanges run in parts serve strided axes only
            if (k->nparts > 1 && m2 == 1) continue;
            const int top = fit_logW(k, 10, p->dtype);
            // widths below 1/16 of the widest that fits are never competitive;
            // of a kernel with exchanges in parts only the two widest are tried
            const int span = k->nparts == 1 ? 4 : 1;
            for (int lw = top; lw >= 0 && top - lw <= span && rc == OFFT_SUCCESS; --lw) {
                if (!tile_fits(k, lw, p->dtype)) continue;
                cur.k[ax] = k;
                cur.logW[ax] = lw;
                float ms = 0.f;
                rc = time_pass(p, cur, ax, buf, s, o.reps, &ms);
                ++timed;
                if (rc == OFFT_SUCCESS && ms < best_ms) {
                    best_ms = ms;
                    best_k = k;
                    best_lw = lw;
                }
            }
        }
        best.k[ax] = best_k;
        best.logW[ax] = best_lw;
    }
    static const int orders[6][3] = {{2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {1, 0, 2}, {0, 2, 1}, {0, 1, 2}};
    PlanChoice winner = best;
    float win_ms = 1e30f;
    for (int i = 0; i < 6 && rc == OFFT_SUCCESS; ++i) {
        PlanChoice c = best;
        for (int j = 0; j < 3; ++j) c.order[j] = orders[i][j];
        float ms = 0.f;
        rc = time_choice(p, c, src, buf, s, o.reps, &ms);
        ++timed;
        if (rc == OFFT_SUCCESS && ms < win_ms) { win_ms = ms; winner = c; }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (src != buf) (void)hipFree(src);
    if (rc != OFFT_SUCCESS) return rc;
    *choice = winner;
    char buf2[160];
    snprintf(buf2, sizeof buf2, "exhaustive: %d timings (per-axis kernels and widths, then 6 orders %s), best %.4f ms",
             timed, o.tune_inplace ? "in place" : "out of place", win_ms);
    p->tune_log = buf2;
    if (o.cache_path) cache_store(o.cache_path, p->dtype, p->dims, p->batch, *choice, win_ms);
    return OFFT_SUCCESS;
}

int select_plan(offt_plan_s* p, const offt_opts& o, PlanChoice* choice) {
    if (o.cache_path && cache_lookup(o.cache_path, p->dtype, p->dims, p->batch, choice) == OFFT_SUCCESS) {
        p->tune_log = "cache";
        return OFFT_SUCCESS;
    }
    if (o.tune == OFFT_TUNE_LEARNED) {
        std::string why;
        if (learned_choice(p->dtype, p->dims, p->batch, o.weights_path, choice, &why) == OFFT_SUCCESS) {
            p->tune_log = "learned";
            return OFFT_SUCCESS;
        }
        // weights missing / unreadable / no feasible prediction: fall back
        const int rc = exhaustive(p, o, choice);
        p->tune_log = "learned-fallback(" + why + ") " + p->tune_log;
        return rc;
    }
    return exhaustive(p, o, choice);
}

}  // namespace offt

extern "C" int offt_tune_table(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch, int reps, void* buf,
                               size_t buf_bytes, void* stream, float* times_ms, int max) {
    using namespace offt;
    int rc = validate_dims(Na, Nb, Nc, dtype, batch);
    const size_t need = (size_t)(Na * Nb * Nc * batch) * elem_size(dtype);
    if (rc == OFFT_SUCCESS && (!buf || buf_bytes < need || reps < 1 || max < 0 || (max > 0 && !times_ms)))
        rc = OFFT_ERR_INVALID_ARG;
    if (rc == OFFT_SUCCESS) rc = check_device();
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    offt_plan_s tmp;
    tmp.kind = 1;
    tmp.dtype = dtype;
    tmp.dims[0] = Na; tmp.dims[1] = Nb; tmp.dims[2] = Nc;
    tmp.batch = batch;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::vector<PlanChoice> cands = candidate_choices(dtype, tmp.dims);
    for (int i = 0; i < std::min((int)cands.size(), max) && rc == OFFT_SUCCESS; ++i)
        rc = time_choice(&tmp, cands[i], buf, buf, s, reps, &times_ms[i]);
    (void)hipStreamSynchronize(s);
    for (void* d : tmp.allocs) (void)hipFree(d);
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    set_error(OFFT_SUCCESS);
    return (int)cands.size();
}

namespace offt {

std::string describe_plan(const offt_plan_s* p) {
    if (p->kind == 2) return describe_many(p);
    return choice_to_string(p->choice, p->dims);
}

}  // namespace offt
