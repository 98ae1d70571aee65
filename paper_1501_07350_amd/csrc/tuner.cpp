// tuner.cpp -- run-time plan selection at plan time, the GPU counterpart of
// the paper's auto-tuning of communication methods (Sec. 3.2.3): every
// candidate plan is executed a few times during initialization and the
// fastest is kept; a plan cache plays the role of the paper's "User-select
// after tuning once".  Candidates: radix sequence (with the parts its LDS
// exchanges run in) and tile width per axis, and the axis order of the
// passes.
//
// Protocol: 1 warm-up + `reps` timed executions per candidate (hipEvents on the
// tuning stream), score = minimum of up to two runs, median of more; ties go
// to the earlier candidate (the heuristic's choices come first).  The data is
// refilled with uniform random values before each candidate (timings on
// all-zero buffers are not representative of real data on this device).
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

std::string cache_key(int dtype, const int64_t dims[3], int64_t batch, int layout) {
    char buf[256];
    snprintf(buf, sizeof buf, "dtype=%d dims=%lldx%lldx%lld batch=%lld dev=%s%s", dtype, (long long)dims[0],
             (long long)dims[1], (long long)dims[2], (long long)batch, device_name().c_str(),
             layout == OFFT_LAYOUT_REVERSED ? " layout=cba" : "");
    return buf;
}

// Parses a plan string of plan p's layout ("<forward>|<backward>" for
// reversed layouts).
static bool plan_from_string(const offt_plan_s* p, const std::string& plan, PlanChoice* c, PlanChoice* cb) {
    const bool reversed = p->layout == OFFT_LAYOUT_REVERSED;
    const size_t bar = plan.find('|');
    if (reversed != (bar != std::string::npos)) return false;
    if (!choice_from_string(plan.substr(0, bar).c_str(), p->dtype, p->dims, c)) return false;
    if (!reversed) return true;
    int64_t rd[3];
    reversed_dims(p->dims, rd);
    return choice_from_string(plan.substr(bar + 1).c_str(), p->dtype, rd, cb);
}

static std::string plan_to_string(const offt_plan_s* p, const PlanChoice& c, const PlanChoice& cb) {
    std::string s = choice_to_string(c, p->dims);
    if (p->layout == OFFT_LAYOUT_REVERSED) {
        int64_t rd[3];
        reversed_dims(p->dims, rd);
        s += "|" + choice_to_string(cb, rd);
    }
    return s;
}

// Returns OFFT_SUCCESS and fills *c (and *cb) when the cache holds a usable entry.
static int cache_lookup(const char* path, const offt_plan_s* p, PlanChoice* c, PlanChoice* cb) {
    std::ifstream f(path);
    if (!f) return OFFT_ERR_IO;
    const std::string key = cache_key(p->dtype, p->dims, p->batch, p->layout);
    std::string line;
    int rc = OFFT_ERR_IO;
    while (std::getline(f, line)) {
        const size_t t1 = line.find('\t');
        if (t1 == std::string::npos || line.compare(0, t1, key) != 0 || t1 != key.size()) continue;
        const size_t t2 = line.find('\t', t1 + 1);
        const std::string plan = line.substr(t1 + 1, t2 == std::string::npos ? std::string::npos : t2 - t1 - 1);
        PlanChoice pc, pcb;
        if (plan_from_string(p, plan, &pc, &pcb)) {
            *c = pc;   // the latest valid entry wins
            if (cb) *cb = pcb;
            rc = OFFT_SUCCESS;
        }
    }
    return rc;
}

static void cache_store(const char* path, const offt_plan_s* p, const PlanChoice& c, const PlanChoice& cb,
                        float ms) {
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    f << cache_key(p->dtype, p->dims, p->batch, p->layout) << '\t' << plan_to_string(p, c, cb) << '\t' << ms
      << '\n';
}

// Times one candidate for a grid of shape `dims` from `src` to `dst` (equal:
// in place), through `work` where a transposing pass needs it.  Returns
// OFFT_SUCCESS and the minimum time in *ms.
// Score of a candidate's timed runs: the minimum of up to two runs (the
// library's default), the median of three or more -- a minimum over many
// runs favours kernels whose time varies from run to run, which then lose
// in steady use.
static float score(std::vector<float>& t) {
    if (t.empty()) return 1e30f;
    std::sort(t.begin(), t.end());
    if (t.size() <= 2) return t[0];
    const size_t m = t.size() / 2;
    return t.size() % 2 ? t[m] : 0.5f * (t[m - 1] + t[m]);
}

// Times a pass list over `nelem` elements (see time_choice).
static int time_passes(offt_plan_s* p, PassPlan* passes, int n, int64_t nelem, void* src, void* dst, void* work,
                       hipStream_t s, int reps, float* ms) {
    for (int i = 0; i < n; ++i)
        if (!passes[i].k) return OFFT_ERR_UNSUPPORTED_SIZE;
    int rc = attach_twiddles(p, passes, n, s);
    if (rc != OFFT_SUCCESS) return rc;
    // fresh random data per candidate: unnormalised transforms repeated in
    // place would otherwise grow the values towards overflow
    if (launch_fill_uniform(src, nelem, p->dtype, 1501, s) != hipSuccess) return OFFT_ERR_HIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return OFFT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return OFFT_ERR_HIP; }
    rc = exec_passes(p, passes, n, src, dst, work, OFFT_FORWARD, s);   // warm-up
    std::vector<float> runs;
    for (int r = 0; r < reps && rc == OFFT_SUCCESS; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) { rc = OFFT_ERR_HIP; break; }
        rc = exec_passes(p, passes, n, src, dst, work, OFFT_FORWARD, s);
        if (rc != OFFT_SUCCESS) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = OFFT_ERR_HIP; break; }
        float t = 0.f;
        if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) { rc = OFFT_ERR_HIP; break; }
        runs.push_back(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = score(runs);
    return rc;
}

int time_choice(offt_plan_s* p, const PlanChoice& c, const int64_t dims[3], void* src, void* dst, void* work,
                hipStream_t s, int reps, float* ms) {
    PassPlan passes[3];
    const int n = build_passes(c, dims, p->batch, passes);
    return time_passes(p, passes, n, dims[0] * dims[1] * dims[2] * p->batch, src, dst, work, s, reps, ms);
}

// Times one axis pass alone: 1 warm-up + reps runs, minimum.  Ordinary
// passes run in place on buf; a transposing pass reads `other` (it never
// runs in place).
static int time_pass(offt_plan_s* p, PassPlan pass, void* buf, void* other, hipStream_t s, int reps, float* ms) {
    if (!pass.k) return OFFT_ERR_UNSUPPORTED_SIZE;
    int rc = attach_twiddles(p, &pass, 1, s);
    if (rc != OFFT_SUCCESS) return rc;
    void* src = pass.mode >= 2 ? other : buf;
    if (!src) return OFFT_ERR_INVALID_ARG;
    if (launch_fill_uniform(src, pass.M1 * pass.M2 * pass.L, p->dtype, 1502, s) != hipSuccess) return OFFT_ERR_HIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return OFFT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return OFFT_ERR_HIP; }
    if (launch_pass(pass, src, buf, 0, 0, 1.0, s) != hipSuccess) rc = OFFT_ERR_HIP;   // warm-up
    std::vector<float> runs;
    for (int r = 0; r < reps && rc == OFFT_SUCCESS; ++r) {
        float t = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess || launch_pass(pass, src, buf, 0, 0, 1.0, s) != hipSuccess ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            rc = OFFT_ERR_HIP;
            break;
        }
        runs.push_back(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = score(runs);
    return rc;
}

namespace {
struct TuneBuffers {
    void* buf = nullptr;    // destination of whole transforms, in-place target of single passes
    void* src = nullptr;    // source of whole transforms (== buf when tuning in place)
    void* work = nullptr;   // reversed layouts: the transposing passes' workspace
};
}  // namespace

// Exhaustive search for one grid shape over a factorised space: the passes
// are independent kernels, so every (radix sequence, threads per line, tile
// width) of each axis is timed as a single pass in every geometry the axis
// can have (on the abc grid; for reversed output also on the cba grid and as
// the transposing pass), and the two fastest kept per axis and geometry
// (the fastest also tried with its tiles in XCD-contiguous order); then the
// heuristic plan and the six pass orders (times the transposing axes) with
// every combination of those kernels are timed as whole transforms.  Ties
// keep the earlier candidate (the heuristic's kernels and order come first).
// kernels per blocked pass tried in a kept block schedule (its axis's
// fastest over the whole grid)
constexpr size_t kBlockKernels = 6;

static int exhaustive_dims(offt_plan_s* p, const offt_opts& o, const int64_t dims[3], bool reversed,
                           const TuneBuffers& B, PlanChoice* choice, float* win_ms_out, int* timed) {
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    const bool rev = reversed && reversal_moves_data(dims);
    const PlanChoice heur = rev ? default_choice_reversed(p->dtype, dims) : default_choice(p->dtype, dims);
    std::vector<int> taxes;   // transposing axes to try
    if (rev) {
        for (int t : {0, 2})
            if (dims[t] > 1) taxes.push_back(t);
    } else {
        taxes.push_back(-1);
    }
    // the two fastest (kernel, width) of each axis and geometry: a pass timed
    // alone can rank near-equal kernels differently than inside the whole
    // transform (what the previous pass leaves in the caches differs), so
    // both go on to the whole-transform stage
    const KernelEntry* best_k[3][3][2] = {};
    int best_lw[3][3][2] = {};
    int best_x[3][3][2] = {};   // XCD-contiguous tile order
    int best_io[3][3][2] = {};  // grid-data access mode (kIoAuto unless a forced mode was faster)
    // every (kernel, width) timed on the input's geometry, fastest first: a
    // pass of a block schedule runs from the Infinity Cache, where kernels
    // rank differently than over the whole grid
    struct Ranked { float ms; const KernelEntry* k; int lw; };
    std::vector<Ranked> ranked[3];
    int rc = OFFT_SUCCESS;
    for (int ax = 0; ax < 3 && rc == OFFT_SUCCESS; ++ax) {
        if (dims[ax] <= 1) continue;
        for (int g = 0; g < 3 && rc == OFFT_SUCCESS; ++g) {
            // geometries the axis can take under some candidate
            bool reachable = false;
            for (int t : taxes)
                reachable = reachable || (g == kGeomTranspose ? t == ax
                                                              : (t < 0 ? g == kGeomNatural : t != ax));
            if (!reachable) continue;
            const PassPlan shape = make_pass(dims, p->batch, ax, g, nullptr, 0);
            // the heuristic's kernel for this geometry first, so ties keep it
            const KernelEntry* hk = nullptr;
            int hlw = 0;
            {
                PlanChoice h = heur;
                if (g == kGeomTranspose) h.tax = ax;
                if (axis_geom(h, ax) == g) { hk = h.k[ax]; hlw = h.logW[ax]; }
            }
            std::vector<const KernelEntry*> ks = kernels_for(p->dtype, (int)dims[ax]);
            std::stable_partition(ks.begin(), ks.end(), [&](const KernelEntry* k) { return k == hk; });
            float best_ms[2] = {1e30f, 1e30f};
            best_k[ax][g][0] = hk;
            best_lw[ax][g][0] = hlw;
            for (const KernelEntry* k : ks) {
                // kernels whose LDS exchanges run in parts serve strided lines
                // (and transposing passes, whose one side is strided)
                if (k->nparts > 1 && shape.M2 == 1) continue;
                if (g == kGeomTranspose && !k->launch_t) continue;
                const int top = fit_logW(k, 10, p->dtype, g);
                // widths below 1/16 of the widest that fits are never competitive;
                // of a kernel with exchanges in parts only the two widest are tried
                const int span = k->nparts == 1 ? 4 : 1;
                for (int lw = top; lw >= 0 && top - lw <= span && rc == OFFT_SUCCESS; --lw) {
                    if (!tile_fits_geom(k, lw, p->dtype, g)) continue;
                    float ms = 0.f;
                    rc = time_pass(p, make_pass(dims, p->batch, ax, g, k, lw), B.buf, B.work, s, o.reps, &ms);
                    ++*timed;
                    if (rc != OFFT_SUCCESS) break;
                    if (g == kGeomNatural) ranked[ax].push_back({ms, k, lw});
                    if (ms < best_ms[0]) {
                        best_ms[1] = best_ms[0];
                        best_k[ax][g][1] = best_k[ax][g][0];
                        best_lw[ax][g][1] = best_lw[ax][g][0];
                        best_ms[0] = ms;
                        best_k[ax][g][0] = k;
                        best_lw[ax][g][0] = lw;
                    } else if (ms < best_ms[1]) {
                        best_ms[1] = ms;
                        best_k[ax][g][1] = k;
                        best_lw[ax][g][1] = lw;
                    }
                }
            }
            // the heuristic's kernel seeded slot 0 before any timing: if it was
            // displaced without being timed faster, slot 1 may still hold it
            if (best_k[ax][g][1] == best_k[ax][g][0] && best_lw[ax][g][1] == best_lw[ax][g][0])
                best_k[ax][g][1] = nullptr;
            // the fastest kernel with its tiles in the other tile order (at
            // 1024^3 the XCD-contiguous order gained 2-5% on every pass with
            // cached accesses, at 512^3 some passes lost), and with the grid
            // data accessed the other way (streaming or cached)
            auto try_variant = [&](int x, int io) {
                if (rc != OFFT_SUCCESS || !best_k[ax][g][0] || best_ms[0] >= 1e30f) return;
                float ms = 0.f;
                rc = time_pass(p, make_pass(dims, p->batch, ax, g, best_k[ax][g][0], best_lw[ax][g][0], x, io),
                               B.buf, B.work, s, o.reps, &ms);
                ++*timed;
                if (rc != OFFT_SUCCESS) return;
                if (ms < best_ms[0]) {
                    best_ms[1] = best_ms[0];
                    best_k[ax][g][1] = best_k[ax][g][0];
                    best_lw[ax][g][1] = best_lw[ax][g][0];
                    best_x[ax][g][1] = best_x[ax][g][0];
                    best_io[ax][g][1] = best_io[ax][g][0];
                    best_ms[0] = ms;
                    best_x[ax][g][0] = x;
                    best_io[ax][g][0] = io;
                } else if (ms < best_ms[1]) {
                    best_ms[1] = ms;
                    best_k[ax][g][1] = best_k[ax][g][0];
                    best_lw[ax][g][1] = best_lw[ax][g][0];
                    best_x[ax][g][1] = x;
                    best_io[ax][g][1] = io;
                }
            };
            if (g != kGeomTranspose) try_variant(1, kIoAuto);
            {
                const int64_t bytes = dims[0] * dims[1] * dims[2] * p->batch * (int64_t)elem_size(p->dtype);
                const int other_io = resolve_stream(kIoAuto, bytes) ? kIoCached : kIoStream;
                try_variant(best_x[ax][g][0], other_io);
            }
        }
    }
    // whole transforms: the heuristic plan itself first (so the choice is
    // never slower than it by this measure), then every order (and
    // transposing axis) with every combination of each axis's two fastest
    // kernels
    static const int orders[6][3] = {{2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {1, 0, 2}, {0, 2, 1}, {0, 1, 2}};
    PlanChoice winner = heur;
    float win_ms = 1e30f;
    if (rc == OFFT_SUCCESS) {
        rc = time_choice(p, heur, dims, B.src, B.buf, B.work, s, o.reps, &win_ms);
        ++*timed;
    }
    for (int t : taxes) {
        for (int i = 0; i < 6 && rc == OFFT_SUCCESS; ++i) {
            for (int combo = 0; combo < 8 && rc == OFFT_SUCCESS; ++combo) {
                PlanChoice c = heur;
                c.tax = t;
                for (int j = 0; j < 3; ++j) c.order[j] = orders[i][j];
                bool valid = true;
                for (int ax = 0; ax < 3; ++ax) {
                    const int pick = (combo >> ax) & 1;
                    if (dims[ax] <= 1) {
                        valid = valid && pick == 0;
                        continue;
                    }
                    const int g = axis_geom(c, ax);
                    valid = valid && best_k[ax][g][pick] != nullptr;
                    c.k[ax] = best_k[ax][g][pick];
                    c.logW[ax] = best_lw[ax][g][pick];
                    c.xcd[ax] = best_x[ax][g][pick];
                    c.io[ax] = best_io[ax][g][pick];
                }
                if (!valid) continue;
                float ms = 0.f;
                rc = time_choice(p, c, dims, B.src, B.buf, B.work, s, o.reps, &ms);
                ++*timed;
                if (rc == OFFT_SUCCESS && ms < win_ms) { win_ms = ms; winner = c; }
            }
        }
    }
    // the winner with one pass's access mode switched, pass by pass, timed as
    // whole transforms: a pass's mode changes what the next pass finds in the
    // caches, which single passes timed alone do not show; a switch is kept
    // when it gains more than 1% (less is within the timing noise)
    const int64_t grid_bytes = dims[0] * dims[1] * dims[2] * p->batch * (int64_t)elem_size(p->dtype);
    for (int ax = 0; ax < 3 && rc == OFFT_SUCCESS; ++ax) {
        if (dims[ax] <= 1 || !winner.k[ax]) continue;
        PlanChoice c = winner;
        c.io[ax] = resolve_stream(winner.io[ax], grid_bytes) ? kIoCached : kIoStream;
        float ms = 0.f;
        rc = time_choice(p, c, dims, B.src, B.buf, B.work, s, o.reps, &ms);
        ++*timed;
        if (rc == OFFT_SUCCESS && ms < 0.99f * win_ms) { win_ms = ms; winner = c; }
    }
    // slab and column-block schedules of grids larger than twice the
    // Infinity Cache: the pass over a first, then the winner's kernels for b
    // and c slab by slab, in both orders, with slabs of 64, 128 and 256 MiB
    // (their passes' access modes resolved per slab); kept when more than 1%
    // faster
    const int64_t plane_bytes = dims[1] * dims[2] * (int64_t)elem_size(p->dtype);
    const int64_t planes = dims[0] * p->batch;
    if (!rev && winner.tax < 0 && dims[0] > 1 && dims[1] * dims[2] > 1 && grid_bytes > 2 * kStreamMinBytes) {
        const PlanChoice base = winner;
        for (int bc = 0; bc < 2 && rc == OFFT_SUCCESS; ++bc) {
            PlanChoice ord = base;
            ord.order[0] = 0;
            ord.order[1] = bc ? 2 : 1;
            ord.order[2] = bc ? 1 : 2;
            ord.io[1] = ord.io[2] = kIoAuto;
            int64_t last = 0;
            for (int64_t mib : {64, 128, 256}) {
                const int64_t slab = std::max<int64_t>(1, (mib << 20) / plane_bytes);
                if (slab >= planes || slab == last || rc != OFFT_SUCCESS) continue;
                last = slab;
                PlanChoice c = ord;
                c.slab = slab;
                float ms = 0.f;
                rc = time_choice(p, c, dims, B.src, B.buf, B.work, s, o.reps, &ms);
                ++*timed;
                if (rc == OFFT_SUCCESS && ms < 0.99f * win_ms) { win_ms = ms; winner = c; }
            }
        }
        // column-block schedules: the pass over c first over the whole grid,
        // then the winner's kernels for b and a on blocks of columns of 64,
        // 128 and 256 MiB, in both orders (the tile widths of both must fit a
        // block)
        const int64_t column_bytes = dims[0] * dims[1] * p->batch * (int64_t)elem_size(p->dtype);
        for (int ba = 0; ba < 2 && rc == OFFT_SUCCESS; ++ba) {
            PlanChoice ord = base;
            ord.slab = 0;
            ord.order[0] = 2;
            ord.order[1] = ba ? 0 : 1;
            ord.order[2] = ba ? 1 : 0;
            ord.io[0] = ord.io[1] = kIoAuto;
            int64_t last = 0;
            for (int64_t mib : {64, 128, 256}) {
                int64_t w = 1;
                while (w * 2 * column_bytes <= (mib << 20)) w *= 2;
                if (w == last || rc != OFFT_SUCCESS) continue;
                last = w;
                PlanChoice c = ord;
                c.col = w;
                if (!col_fits(c, dims, true)) continue;
                float ms = 0.f;
                rc = time_choice(p, c, dims, B.src, B.buf, B.work, s, o.reps, &ms);
                ++*timed;
                if (rc == OFFT_SUCCESS && ms < 0.99f * win_ms) { win_ms = ms; winner = c; }
            }
        }
        // a kept schedule, its blocked passes refined in place: each with its
        // other fast kernel, with the other tile order and with the other
        // access mode (what a pass finds in the cache, how many tiles a block
        // holds and what its stores leave in the cache for the next block
        // differ from the whole-grid passes they were ranked on)
        const int64_t block_bytes = winner.slab > 0 ? std::min(winner.slab, planes) * plane_bytes
                                                    : winner.col * column_bytes;
        for (int ax = 0; ax < 3 && (winner.slab > 0 || winner.col > 0) && rc == OFFT_SUCCESS; ++ax) {
            if (dims[ax] <= 1 || ax == (winner.slab > 0 ? 0 : 2)) continue;   // the whole-grid pass
            const int g = axis_geom(winner, ax);
            std::stable_sort(ranked[ax].begin(), ranked[ax].end(),
                             [](const Ranked& x, const Ranked& y) { return x.ms < y.ms; });
            const int nk = (int)std::min<size_t>(ranked[ax].size(), kBlockKernels);
            for (int variant = -nk; variant < 3 && rc == OFFT_SUCCESS; ++variant) {
                PlanChoice c = winner;
                if (variant < 0) {
                    // one of the axis's fastest whole-grid kernels, the winner's own aside
                    const Ranked& r = ranked[ax][nk + variant];
                    if (r.k == winner.k[ax] && r.lw == winner.logW[ax]) continue;
                    c.k[ax] = r.k;
                    c.logW[ax] = r.lw;
                } else if (variant == 0) {
                    const int other = best_k[ax][g][0] == winner.k[ax] && best_lw[ax][g][0] == winner.logW[ax] ? 1 : 0;
                    if (!best_k[ax][g][other]) continue;
                    c.k[ax] = best_k[ax][g][other];
                    c.logW[ax] = best_lw[ax][g][other];
                    c.xcd[ax] = best_x[ax][g][other];
                } else if (variant == 1) {
                    c.xcd[ax] = !winner.xcd[ax];
                } else {
                    c.io[ax] = resolve_stream(winner.io[ax], block_bytes) ? kIoCached : kIoStream;
                }
                if (!col_fits(c, dims, true)) continue;
                float ms = 0.f;
                rc = time_choice(p, c, dims, B.src, B.buf, B.work, s, o.reps, &ms);
                ++*timed;
                if (rc == OFFT_SUCCESS && ms < 0.99f * win_ms) { win_ms = ms; winner = c; }
            }
        }
    }
    if (rc != OFFT_SUCCESS) return rc;
    *choice = winner;
    *win_ms_out = win_ms;
    return OFFT_SUCCESS;
}

static int exhaustive(offt_plan_s* p, const offt_opts& o, PlanChoice* choice, PlanChoice* choice_b) {
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    const bool reversed = p->layout == OFFT_LAYOUT_REVERSED;
    const size_t bytes = (size_t)(p->dims[0] * p->dims[1] * p->dims[2] * p->batch) * elem_size(p->dtype);
    // whole transforms are timed out of place (src -> buf) unless the caller
    // tunes for in-place use; single passes run in place on buf (transposing
    // ones from work to buf)
    TuneBuffers B;
    int rc = OFFT_SUCCESS;
    auto alloc = [&](void** d) {
        if (rc == OFFT_SUCCESS && hipMalloc(d, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *d = nullptr;
            rc = OFFT_ERR_OUT_OF_MEMORY;
        }
    };
    alloc(&B.buf);
    if (o.tune_inplace) B.src = B.buf;
    else alloc(&B.src);
    if (reversed && reversal_moves_data(p->dims)) alloc(&B.work);
    int timed = 0;
    float ms = 0.f, ms_b = 0.f;
    if (rc == OFFT_SUCCESS) rc = exhaustive_dims(p, o, p->dims, reversed, B, choice, &ms, &timed);
    if (rc == OFFT_SUCCESS && reversed) {
        int64_t rd[3];
        reversed_dims(p->dims, rd);
        if (rd[0] == p->dims[0]) {
            *choice_b = *choice;   // Na == Nc: the backward shape is the same
            ms_b = ms;
        } else {
            rc = exhaustive_dims(p, o, rd, true, B, choice_b, &ms_b, &timed);
        }
    }
    (void)hipStreamSynchronize(s);
    if (B.buf) (void)hipFree(B.buf);
    if (B.src && B.src != B.buf) (void)hipFree(B.src);
    if (B.work) (void)hipFree(B.work);
    if (rc != OFFT_SUCCESS) return rc;
    char buf2[200];
    if (reversed)
        snprintf(buf2, sizeof buf2,
                 "exhaustive: %d timings (per-axis kernels and widths per geometry, then orders and transposing "
                 "axes %s), best %.4f ms forward, %.4f ms backward",
                 timed, o.tune_inplace ? "in place" : "out of place", ms, ms_b);
    else
        snprintf(buf2, sizeof buf2,
                 "exhaustive: %d timings (per-axis kernels and widths, then 6 orders %s), best %.4f ms", timed,
                 o.tune_inplace ? "in place" : "out of place", ms);
    p->tune_log = buf2;
    if (o.cache_path) cache_store(o.cache_path, p, *choice, reversed ? *choice_b : *choice, ms);
    return OFFT_SUCCESS;
}

int select_plan(offt_plan_s* p, const offt_opts& o, PlanChoice* choice, PlanChoice* choice_b) {
    if (o.cache_path && cache_lookup(o.cache_path, p, choice, choice_b) == OFFT_SUCCESS) {
        p->tune_log = "cache";
        return OFFT_SUCCESS;
    }
    if (o.tune == OFFT_TUNE_LEARNED && p->layout == OFFT_LAYOUT_REVERSED) {
        // the learned selector ranks natural-layout candidates only
        const int rc = exhaustive(p, o, choice, choice_b);
        p->tune_log = "learned-fallback(reversed layout) " + p->tune_log;
        return rc;
    }
    if (o.tune == OFFT_TUNE_LEARNED) {
        std::string why;
        if (learned_choice(p->dtype, p->dims, p->batch, o.weights_path, choice, &why) == OFFT_SUCCESS) {
            p->tune_log = "learned";
            return OFFT_SUCCESS;
        }
        // weights missing / unreadable / no feasible prediction: fall back
        const int rc = exhaustive(p, o, choice, choice_b);
        p->tune_log = "learned-fallback(" + why + ") " + p->tune_log;
        return rc;
    }
    return exhaustive(p, o, choice, choice_b);
}

// ---- grids of 4 and 5 axes -----------------------------------------------------

static std::string cache_key_nd(const offt_plan_s* p) {
    std::ostringstream os;
    os << "dtype=" << p->dtype << " dims=";
    for (int i = 0; i < p->ndim; ++i) os << (i ? "x" : "") << p->nd_dims[i];
    os << " batch=" << p->batch << " dev=" << device_name();
    return os.str();
}

// Exhaustive search for a D-dimensional grid: every kernel and width of each
// axis timed as a single pass (its geometry does not depend on the order),
// the two fastest kept per axis, then every order of the passes over the
// axes longer than 1 timed as whole transforms with the fastest kernels --
// up to 5! = 120 orders, the counterpart of the paper's analysis of all
// transpose orders -- and the winning order with every mix of the two.
// Ties keep the earlier candidate (the heuristic's kernels, then its order,
// first).
static int exhaustive_nd(offt_plan_s* p, const offt_opts& o, NdChoice* choice, float* win_ms, int* timed) {
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    const int64_t nelem = p->grid_elems() * p->batch;
    const size_t bytes = (size_t)nelem * elem_size(p->dtype);
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
    const int D = p->ndim;
    const int64_t* dims = p->nd_dims;
    NdChoice best = default_choice_nd(p->dtype, D, dims);
    // runner-up (kernel, width) per axis, tried with the winning order at the end
    const KernelEntry* second_k[kMaxDims] = {};
    int second_lw[kMaxDims] = {};
    int second_x[kMaxDims] = {};
    int second_io[kMaxDims] = {};
    int rc = OFFT_SUCCESS;
    for (int ax = 0; ax < D && rc == OFFT_SUCCESS; ++ax) {
        if (dims[ax] <= 1) continue;
        const bool strided = make_pass_nd(D, dims, 1, ax, nullptr, 0).M2 > 1;
        std::vector<const KernelEntry*> ks = kernels_for(p->dtype, (int)dims[ax]);
        std::stable_partition(ks.begin(), ks.end(), [&](const KernelEntry* k) { return k == best.k[ax]; });
        float best_ms = 1e30f, second_ms = 1e30f;
        const KernelEntry* bk = best.k[ax];
        int blw = best.logW[ax];
        for (const KernelEntry* k : ks) {
            if (k->nparts > 1 && !strided) continue;
            const int top = fit_logW(k, 10, p->dtype);
            const int span = k->nparts == 1 ? 4 : 1;
            for (int lw = top; lw >= 0 && top - lw <= span && rc == OFFT_SUCCESS; --lw) {
                if (!tile_fits(k, lw, p->dtype)) continue;
                float ms = 0.f;
                rc = time_pass(p, make_pass_nd(D, dims, p->batch, ax, k, lw), buf, nullptr, s, o.reps, &ms);
                ++*timed;
                if (rc != OFFT_SUCCESS) break;
                if (ms < best_ms) {
                    if (best_ms < 1e30f) {
                        second_ms = best_ms;
                        second_k[ax] = bk;
                        second_lw[ax] = blw;
                    }
                    best_ms = ms;
                    bk = k;
                    blw = lw;
                } else if (ms < second_ms) {
                    second_ms = ms;
                    second_k[ax] = k;
                    second_lw[ax] = lw;
                }
            }
        }
        best.k[ax] = bk;
        best.logW[ax] = blw;
        // the fastest kernel with its tiles in XCD-contiguous order, then
        // with the grid data accessed the other way (streaming or cached)
        auto try_variant = [&](int x, int io) {
            if (rc != OFFT_SUCCESS || !bk || best_ms >= 1e30f) return;
            float ms = 0.f;
            rc = time_pass(p, make_pass_nd(D, dims, p->batch, ax, bk, blw, x, io), buf, nullptr, s, o.reps, &ms);
            ++*timed;
            if (rc != OFFT_SUCCESS) return;
            if (ms < best_ms) {
                second_ms = best_ms;
                second_k[ax] = bk;
                second_lw[ax] = blw;
                second_x[ax] = best.xcd[ax];
                second_io[ax] = best.io[ax];
                best_ms = ms;
                best.xcd[ax] = x;
                best.io[ax] = io;
            } else if (ms < second_ms) {
                second_ms = ms;
                second_k[ax] = bk;
                second_lw[ax] = blw;
                second_x[ax] = x;
                second_io[ax] = io;
            }
        };
        best.xcd[ax] = 0;
        best.io[ax] = kIoAuto;
        try_variant(1, kIoAuto);
        try_variant(best.xcd[ax], resolve_stream(kIoAuto, nelem * (int64_t)elem_size(p->dtype)) ? kIoCached : kIoStream);
    }
    // orders: the heuristic's first, then every other permutation of the
    // transformed axes (unit axes keep their slots at the end)
    std::vector<int> axes;
    for (int i = 0; i < D; ++i)
        if (dims[best.order[i]] > 1) axes.push_back(best.order[i]);
    std::vector<std::vector<int>> orders{axes};
    std::vector<int> perm = axes;
    std::sort(perm.begin(), perm.end());
    do {
        if (perm != axes) orders.push_back(perm);
    } while (std::next_permutation(perm.begin(), perm.end()));
    // the heuristic plan itself first, then every order with the fastest kernels
    NdChoice winner = default_choice_nd(p->dtype, D, dims);
    float wms = 1e30f;
    if (rc == OFFT_SUCCESS) {
        PassPlan passes[kMaxDims];
        const int n = build_passes_nd(winner, dims, p->batch, passes);
        rc = time_passes(p, passes, n, nelem, src, buf, nullptr, s, o.reps, &wms);
        ++*timed;
    }
    for (size_t oi = 0; oi < orders.size() && rc == OFFT_SUCCESS; ++oi) {
        NdChoice c = best;
        int pos = 0;
        for (int ax : orders[oi]) c.order[pos++] = ax;
        for (int i = 0; i < D; ++i)
            if (dims[i] <= 1) c.order[pos++] = i;
        PassPlan passes[kMaxDims];
        const int n = build_passes_nd(c, dims, p->batch, passes);
        float ms = 0.f;
        rc = time_passes(p, passes, n, nelem, src, buf, nullptr, s, o.reps, &ms);
        ++*timed;
        if (rc == OFFT_SUCCESS && ms < wms) { wms = ms; winner = c; }
    }
    // with the winning order, every combination of each axis's two fastest
    // kernels (a pass timed alone can rank near-equal kernels differently
    // than inside the whole transform)
    const NdChoice base = winner;
    for (int combo = 1; combo < (1 << D) && rc == OFFT_SUCCESS; ++combo) {
        NdChoice c = base;
        bool valid = true;
        for (int ax = 0; ax < D; ++ax) {
            if (!((combo >> ax) & 1)) continue;
            valid = valid && dims[ax] > 1 && second_k[ax] != nullptr;
            c.k[ax] = second_k[ax];
            c.logW[ax] = second_lw[ax];
            c.xcd[ax] = second_x[ax];
            c.io[ax] = second_io[ax];
        }
        if (!valid) continue;
        PassPlan passes[kMaxDims];
        const int n = build_passes_nd(c, dims, p->batch, passes);
        float ms = 0.f;
        rc = time_passes(p, passes, n, nelem, src, buf, nullptr, s, o.reps, &ms);
        ++*timed;
        if (rc == OFFT_SUCCESS && ms < wms) { wms = ms; winner = c; }
    }
    // slab schedules of grids larger than twice the Infinity Cache, as for
    // three axes: the pass over the first axis first, then the other passes
    // slab by slab, in the winner's order or from the contiguous axis down,
    // with slabs of 64, 128 and 256 MiB; kept when more than 1% faster
    int64_t rest = 1;
    for (int ax = 1; ax < D; ++ax) rest *= dims[ax];
    const int64_t es = (int64_t)elem_size(p->dtype);
    const int64_t planes = dims[0] * p->batch;
    if (D >= 2 && dims[0] > 1 && rest > 1 && nelem * es > 2 * kStreamMinBytes) {
        const NdChoice top = winner;
        for (int variant = 0; variant < 2 && rc == OFFT_SUCCESS; ++variant) {
            NdChoice ord = top;
            int pos = 0;
            ord.order[pos++] = 0;
            if (variant == 0) {
                for (int i = 0; i < D; ++i)
                    if (top.order[i] != 0) ord.order[pos++] = top.order[i];
            } else {
                for (int ax = D - 1; ax >= 1; --ax) ord.order[pos++] = ax;
            }
            for (int ax = 1; ax < D; ++ax) ord.io[ax] = kIoAuto;
            int64_t last = 0;
            for (int64_t mib : {64, 128, 256}) {
                const int64_t slab = std::max<int64_t>(1, (mib << 20) / (rest * es));
                if (slab >= planes || slab == last || rc != OFFT_SUCCESS) continue;
                last = slab;
                NdChoice c = ord;
                c.slab = slab;
                PassPlan passes[kMaxDims];
                const int n = build_passes_nd(c, dims, p->batch, passes);
                float ms = 0.f;
                rc = time_passes(p, passes, n, nelem, src, buf, nullptr, s, o.reps, &ms);
                ++*timed;
                if (rc == OFFT_SUCCESS && ms < 0.99f * wms) { wms = ms; winner = c; }
            }
        }
        // a kept schedule: each blocked pass with the other access mode
        // (streaming stores of a block's last passes leave the cache to the
        // next block)
        const int64_t block_bytes = std::min(winner.slab, planes) * rest * es;
        for (int ax = 1; ax < D && winner.slab > 0 && rc == OFFT_SUCCESS; ++ax) {
            if (dims[ax] <= 1) continue;
            NdChoice c = winner;
            c.io[ax] = resolve_stream(winner.io[ax], block_bytes) ? kIoCached : kIoStream;
            PassPlan passes[kMaxDims];
            const int n = build_passes_nd(c, dims, p->batch, passes);
            float ms = 0.f;
            rc = time_passes(p, passes, n, nelem, src, buf, nullptr, s, o.reps, &ms);
            ++*timed;
            if (rc == OFFT_SUCCESS && ms < 0.99f * wms) { wms = ms; winner = c; }
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (src != buf) (void)hipFree(src);
    if (rc != OFFT_SUCCESS) return rc;
    *choice = winner;
    *win_ms = wms;
    return OFFT_SUCCESS;
}

int select_plan_nd(offt_plan_s* p, const offt_opts& o, NdChoice* choice) {
    const std::string key = cache_key_nd(p);
    if (o.cache_path) {
        std::ifstream f(o.cache_path);
        std::string line;
        bool hit = false;
        while (f && std::getline(f, line)) {
            const size_t t1 = line.find('\t');
            if (t1 == std::string::npos || t1 != key.size() || line.compare(0, t1, key) != 0) continue;
            const size_t t2 = line.find('\t', t1 + 1);
            const std::string plan = line.substr(t1 + 1, t2 == std::string::npos ? std::string::npos : t2 - t1 - 1);
            NdChoice c;
            if (nd_choice_from_string(plan.c_str(), p->dtype, p->ndim, p->nd_dims, &c)) {
                *choice = c;   // the latest valid entry wins
                hit = true;
            }
        }
        if (hit) {
            p->tune_log = "cache";
            return OFFT_SUCCESS;
        }
    }
    int timed = 0;
    float ms = 0.f;
    const int rc = exhaustive_nd(p, o, choice, &ms, &timed);
    if (rc != OFFT_SUCCESS) return rc;
    char buf[200];
    snprintf(buf, sizeof buf, "%sexhaustive: %d timings (per-axis kernels and widths, then every pass order %s), "
             "best %.4f ms", o.tune == OFFT_TUNE_LEARNED ? "learned-fallback(4-D/5-D grid) " : "", timed,
             o.tune_inplace ? "in place" : "out of place", ms);
    p->tune_log = buf;
    if (o.cache_path) {
        std::ofstream f(o.cache_path, std::ios::app);
        if (f) f << key << '\t' << nd_choice_to_string(*choice, p->nd_dims) << '\t' << ms << '\n';
    }
    return OFFT_SUCCESS;
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
    const std::vector<PlanChoice> cands = selector_candidates(dtype, tmp.dims, batch);
    for (int i = 0; i < std::min((int)cands.size(), max) && rc == OFFT_SUCCESS; ++i)
        rc = time_choice(&tmp, cands[i], tmp.dims, buf, buf, nullptr, s, reps, &times_ms[i]);
    (void)hipStreamSynchronize(s);
    for (void* d : tmp.allocs) (void)hipFree(d);
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    set_error(OFFT_SUCCESS);
    return (int)cands.size();
}

namespace offt {

std::string describe_plan(const offt_plan_s* p) {
    if (p->kind == 2) return describe_many(p);
    if (p->kind == 4) return describe_dist(p);
    if (p->kind == 3) return nd_choice_to_string(p->ndc, p->nd_dims);
    return plan_to_string(p, p->choice, p->choice_b);
}

}  // namespace offt
