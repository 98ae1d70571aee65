// api.cpp -- the C ABI: plan (initialization), exec (execution), destroy
// (finalization), following the three phases of the paper's calculation flow
// (Sec. 3.1.1).  All device allocations happen at plan time (Sec. 3.2.4);
// exec only launches kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/offt.h"
#include "offt_internal.h"
#include "plan_impl.h"

namespace offt {

static thread_local int g_last_error = OFFT_SUCCESS;
void set_error(int code) { g_last_error = code; }

int check_device() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return OFFT_ERR_NO_DEVICE;
    }
    return OFFT_SUCCESS;
}

int validate_dims(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch) {
    if (dtype != OFFT_C2C_F64 && dtype != OFFT_C2C_F32) return OFFT_ERR_INVALID_ARG;
    if (Na < 1 || Nb < 1 || Nc < 1 || batch < 1) return OFFT_ERR_INVALID_ARG;
    const int64_t d[3] = {Na, Nb, Nc};
    for (int64_t n : d)
        if (!smooth235(n) || n > OFFT_MAX_AXIS) return OFFT_ERR_UNSUPPORTED_SIZE;
    // batch * N * elem must not overflow a signed 64-bit byte count
    const long double bytes = (long double)Na * Nb * Nc * batch * elem_size(dtype);
    if (bytes > 9.0e18L) return OFFT_ERR_INVALID_ARG;
    return OFFT_SUCCESS;
}

// Allocate and fill the twiddle table for every distinct pass length.
int attach_twiddles(offt_plan_s* p, PassPlan* passes, int npass, hipStream_t s) {
    for (int i = 0; i < npass; ++i) {
        const int L = passes[i].L;
        auto it = p->tw.find(L);
        if (it == p->tw.end()) {
            void* d = nullptr;
            const size_t bytes = (size_t)L * elem_size(p->dtype);
            if (hipMalloc(&d, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return OFFT_ERR_OUT_OF_MEMORY;
            }
            p->allocs.push_back(d);
            p->alloc_bytes.push_back(bytes);
            if (launch_twiddles(d, L, p->dtype, s) != hipSuccess) return OFFT_ERR_HIP;
            it = p->tw.emplace(L, d).first;
        }
        passes[i].tw = it->second;
    }
    return OFFT_SUCCESS;
}

int set_choice(offt_plan_s* p, const PlanChoice& c, hipStream_t s) {
    p->choice = c;
    p->npass = build_passes(c, p->dims, p->batch, p->passes);
    for (int i = 0; i < p->npass; ++i)
        if (!p->passes[i].k) return OFFT_ERR_UNSUPPORTED_SIZE;
    return attach_twiddles(p, p->passes, p->npass, s);
}

void reversed_dims(const int64_t dims[3], int64_t out[3]) {
    out[0] = dims[2];
    out[1] = dims[1];
    out[2] = dims[0];
}

int set_choice_b(offt_plan_s* p, const PlanChoice& c, hipStream_t s) {
    int64_t rd[3];
    reversed_dims(p->dims, rd);
    p->choice_b = c;
    const int n = build_passes(c, rd, p->batch, p->passes_b);
    if (n != p->npass) return OFFT_ERR_BAD_PLAN;
    for (int i = 0; i < n; ++i)
        if (!p->passes_b[i].k) return OFFT_ERR_UNSUPPORTED_SIZE;
    return attach_twiddles(p, p->passes_b, n, s);
}

const PassPlan* dir_passes(const offt_plan_s* p, int dir) {
    return (p->layout == OFFT_LAYOUT_REVERSED && dir > 0) ? p->passes_b : p->passes;
}

int exec_passes(const offt_plan_s* p, const PassPlan* passes, int npass, const void* in, void* out,
                void* work, int dir, hipStream_t s, int normalize, int i0, int i1) {
    const int64_t N = p->grid_elems();
    if (i1 < 0) i1 = npass;
    if (npass == 0) {
        if (in != out) {
            const size_t bytes = (size_t)(N * p->batch) * elem_size(p->dtype);
            if (hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return OFFT_ERR_HIP;
        }
        return OFFT_SUCCESS;
    }
    const bool bwd = dir > 0;
    const int norm = normalize < 0 ? p->normalize : normalize;
    const size_t es = elem_size(p->dtype);
    // pass i (whole grid, the planes of one slab at element offset off, or
    // one column block)
    auto launch = [&](int i, const PassPlan& q, int64_t off) {
        const bool last = i == npass - 1;
        const double scale = (bwd && last && norm) ? 1.0 / (double)N : 1.0;
        const void* src = nullptr;
        void* dst = nullptr;
        if (!pass_io(passes, npass, i, in, out, work, &src, &dst)) return OFFT_ERR_BAD_PLAN;
        if (launch_pass(q, static_cast<const char*>(src) + off * es, static_cast<char*>(dst) + off * es,
                        bwd && i == 0, bwd && last, scale, s) != hipSuccess)
            return OFFT_ERR_HIP;
        return OFFT_SUCCESS;
    };
    // passes before the block schedule (all of them without one) over the
    // whole grid, then the schedule: every remaining pass of one slab (or
    // column block) before the next
    const int first_slab = slab_start(passes, npass);
    for (int i = i0; i < std::min(i1, first_slab); ++i) {
        const int rc = launch(i, passes[i], 0);
        if (rc != OFFT_SUCCESS) return rc;
    }
    const int j0 = std::max(i0, first_slab);
    if (j0 >= i1) return OFFT_SUCCESS;
    const PassPlan& sp = passes[first_slab];
    if (sp.col > 0) {
        // column blocks: every remaining pass of one block before the next
        for (int64_t c0 = 0; c0 < sp.ncol; c0 += sp.col) {
            for (int i = j0; i < i1; ++i) {
                const int rc = launch(i, col_pass(passes[i], c0), 0);
                if (rc != OFFT_SUCCESS) return rc;
            }
        }
        return OFFT_SUCCESS;
    }
    for (int64_t p0 = 0; p0 < sp.planes; p0 += sp.slab) {
        const int64_t np = std::min(sp.slab, sp.planes - p0);
        for (int i = j0; i < i1; ++i) {
            int64_t off = 0;
            const PassPlan q = slab_pass(passes[i], p0, np, &off);
            const int rc = launch(i, q, off);
            if (rc != OFFT_SUCCESS) return rc;
        }
    }
    return OFFT_SUCCESS;
}

}  // namespace offt

int64_t offt_plan_s::grid_elems() const {
    if (kind == 3) {
        int64_t n = 1;
        for (int i = 0; i < ndim; ++i) n *= nd_dims[i];
        return n;
    }
    return dims[0] * dims[1] * dims[2];
}

int64_t offt_plan_s::workspace_bytes() const {
    int64_t b = 0;
    for (size_t x : alloc_bytes) b += (int64_t)x;
    return b;
}

namespace offt {

void free_plan(offt_plan_s* p) {
    if (!p) return;
    release_many(p);
    release_dist(p);
    for (int d = 0; d < 2; ++d) {
        if (p->gexec[d]) (void)hipGraphExecDestroy(p->gexec[d]);
        if (p->graph[d]) (void)hipGraphDestroy(p->graph[d]);
    }
    if (p->cap) (void)hipStreamDestroy(p->cap);
    for (void* d : p->allocs) (void)hipFree(d);
    delete p;
}

}  // namespace offt

using namespace offt;

extern "C" {

void offt_opts_default(offt_opts* o) {
    if (!o) return;
    o->tune = OFFT_TUNE_NONE;
    o->reps = 2;
    o->normalize_inverse = 0;
    o->forced_plan = nullptr;
    o->cache_path = nullptr;
    o->weights_path = nullptr;
    o->stream = nullptr;
    o->tune_inplace = 0;
    o->use_graph = 0;
    o->layout = OFFT_LAYOUT_NATURAL;
}

int offt_last_error(void) { return g_last_error; }

const char* offt_error_string(int code) {
    switch (code) {
        case OFFT_SUCCESS: return "success";
        case OFFT_ERR_INVALID_ARG: return "invalid argument";
        case OFFT_ERR_UNSUPPORTED_SIZE: return "unsupported size (axis not 2/3/5-smooth or too long)";
        case OFFT_ERR_OUT_OF_MEMORY: return "device out of memory";
        case OFFT_ERR_NO_DEVICE: return "no HIP device";
        case OFFT_ERR_HIP: return "HIP runtime error";
        case OFFT_ERR_BAD_PLAN: return "bad plan";
        case OFFT_ERR_IO: return "plan cache or weights file I/O error";
        default: return "unknown error";
    }
}

offt_plan_t offt_plan(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch) {
    return offt_plan_ex(Na, Nb, Nc, dtype, batch, nullptr);
}

offt_plan_t offt_plan_ex(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch,
                         const offt_opts* o) {
    offt_opts opts;
    offt_opts_default(&opts);
    if (o) opts = *o;
    int rc = validate_dims(Na, Nb, Nc, dtype, batch);
    if (rc == OFFT_SUCCESS && (opts.tune < OFFT_TUNE_NONE || opts.tune > OFFT_TUNE_FORCED))
        rc = OFFT_ERR_INVALID_ARG;
    if (rc == OFFT_SUCCESS && opts.tune == OFFT_TUNE_FORCED && !opts.forced_plan)
        rc = OFFT_ERR_INVALID_ARG;
    if (rc == OFFT_SUCCESS && (opts.reps < 1 || (opts.use_graph != 0 && opts.use_graph != 1)))
        rc = OFFT_ERR_INVALID_ARG;
    if (rc == OFFT_SUCCESS && opts.layout != OFFT_LAYOUT_NATURAL && opts.layout != OFFT_LAYOUT_REVERSED)
        rc = OFFT_ERR_INVALID_ARG;
    if (rc != OFFT_SUCCESS) { set_error(rc); return nullptr; }
    const int64_t dims[3] = {Na, Nb, Nc};
    int64_t rdims[3];
    reversed_dims(dims, rdims);
    const bool reversed = opts.layout == OFFT_LAYOUT_REVERSED;
    PlanChoice forced, forced_b;
    if (opts.tune == OFFT_TUNE_FORCED) {
        // reversed layouts: "<forward plan>|<backward plan>", the backward
        // half naming the axes of the cba input; without '|' the backward
        // plan is the heuristic's
        const std::string fp(opts.forced_plan);
        const size_t bar = fp.find('|');
        bool ok = choice_from_string(fp.substr(0, bar).c_str(), dtype, dims, &forced);
        if (ok && reversed) {
            if (bar != std::string::npos)
                ok = choice_from_string(fp.substr(bar + 1).c_str(), dtype, rdims, &forced_b);
            else
                forced_b = default_choice_reversed(dtype, rdims);
        }
        // a plan string must give the output order the layout asks for
        if (ok && (forced.tax >= 0) != (reversed && reversal_moves_data(dims))) ok = false;
        if (ok && reversed && (forced_b.tax >= 0) != reversal_moves_data(dims)) ok = false;
        if (ok && !reversed && bar != std::string::npos) ok = false;
        if (!ok) {
            set_error(OFFT_ERR_BAD_PLAN);
            return nullptr;
        }
    }
    rc = check_device();
    if (rc != OFFT_SUCCESS) { set_error(rc); return nullptr; }

    offt_plan_s* p = new offt_plan_s();
    p->kind = 1;
    p->dtype = dtype;
    p->dims[0] = Na; p->dims[1] = Nb; p->dims[2] = Nc;
    p->batch = batch;
    p->normalize = opts.normalize_inverse ? 1 : 0;
    p->layout = opts.layout;
    hipStream_t s = static_cast<hipStream_t>(opts.stream);

    PlanChoice choice = reversed ? default_choice_reversed(dtype, dims) : default_choice(dtype, dims);
    PlanChoice choice_b = reversed ? default_choice_reversed(dtype, rdims) : choice;
    if (opts.tune == OFFT_TUNE_FORCED) {
        choice = forced;
        choice_b = forced_b;
    } else if (opts.tune == OFFT_TUNE_EXHAUSTIVE || opts.tune == OFFT_TUNE_LEARNED) {
        rc = select_plan(p, opts, &choice, &choice_b);
        if (rc != OFFT_SUCCESS) { free_plan(p); set_error(rc); return nullptr; }
    }
    rc = set_choice(p, choice, s);
    if (rc == OFFT_SUCCESS && reversed) rc = set_choice_b(p, choice_b, s);
    if (rc == OFFT_SUCCESS && reversed && reversal_moves_data(dims)) {
        // the workspace of the transposing passes: one batch of grids
        const size_t bytes = (size_t)(Na * Nb * Nc * batch) * elem_size(dtype);
        if (hipMalloc(&p->work, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p->work = nullptr;
            rc = OFFT_ERR_OUT_OF_MEMORY;
        } else {
            p->allocs.push_back(p->work);
            p->alloc_bytes.push_back(bytes);
        }
    }
    if (rc == OFFT_SUCCESS && hipStreamSynchronize(s) != hipSuccess) rc = OFFT_ERR_HIP;
    // the capture stream of use_graph (default priority, non-blocking)
    p->use_graph = opts.use_graph;
    if (rc == OFFT_SUCCESS && p->use_graph && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        p->cap = nullptr;
        rc = OFFT_ERR_HIP;
    }
    if (rc != OFFT_SUCCESS) { free_plan(p); set_error(rc); return nullptr; }
    set_error(OFFT_SUCCESS);
    return p;
}

// Grids of 1 to 5 axes.  Up to three axes are the three-dimensional plan of
// the shape padded with leading unit axes; 4 and 5 axes get a kind-3 plan
// over the same pass kernels.
static int validate_nd(int ndim, const int64_t* dims, int dtype, int64_t batch) {
    if (ndim < 1 || ndim > OFFT_MAX_DIMS || !dims) return OFFT_ERR_INVALID_ARG;
    if (dtype != OFFT_C2C_F64 && dtype != OFFT_C2C_F32) return OFFT_ERR_INVALID_ARG;
    if (batch < 1) return OFFT_ERR_INVALID_ARG;
    long double bytes = (long double)batch * elem_size(dtype);
    for (int i = 0; i < ndim; ++i) {
        if (dims[i] < 1) return OFFT_ERR_INVALID_ARG;
        if (!smooth235(dims[i]) || dims[i] > OFFT_MAX_AXIS) return OFFT_ERR_UNSUPPORTED_SIZE;
        bytes *= (long double)dims[i];
    }
    if (bytes > 9.0e18L) return OFFT_ERR_INVALID_ARG;
    return OFFT_SUCCESS;
}

offt_plan_t offt_plan_nd(int ndim, const int64_t* dims, int dtype, int64_t batch, const offt_opts* o) {
    int rc = validate_nd(ndim, dims, dtype, batch);
    if (rc != OFFT_SUCCESS) { set_error(rc); return nullptr; }
    if (ndim <= 3) {
        int64_t d3[3] = {1, 1, 1};
        for (int i = 0; i < ndim; ++i) d3[3 - ndim + i] = dims[i];
        return offt_plan_ex(d3[0], d3[1], d3[2], dtype, batch, o);
    }
    offt_opts opts;
    offt_opts_default(&opts);
    if (o) opts = *o;
    if (opts.tune < OFFT_TUNE_NONE || opts.tune > OFFT_TUNE_FORCED ||
        (opts.tune == OFFT_TUNE_FORCED && !opts.forced_plan) || opts.reps < 1 ||
        (opts.use_graph != 0 && opts.use_graph != 1) || opts.layout != OFFT_LAYOUT_NATURAL) {
        set_error(OFFT_ERR_INVALID_ARG);
        return nullptr;
    }
    NdChoice choice = default_choice_nd(dtype, ndim, dims);
    if (opts.tune == OFFT_TUNE_FORCED && !nd_choice_from_string(opts.forced_plan, dtype, ndim, dims, &choice)) {
        set_error(OFFT_ERR_BAD_PLAN);
        return nullptr;
    }
    rc = check_device();
    if (rc != OFFT_SUCCESS) { set_error(rc); return nullptr; }
    offt_plan_s* p = new offt_plan_s();
    p->kind = 3;
    p->dtype = dtype;
    p->ndim = ndim;
    for (int i = 0; i < ndim; ++i) p->nd_dims[i] = dims[i];
    p->batch = batch;
    p->normalize = opts.normalize_inverse ? 1 : 0;
    hipStream_t s = static_cast<hipStream_t>(opts.stream);
    if (opts.tune == OFFT_TUNE_EXHAUSTIVE || opts.tune == OFFT_TUNE_LEARNED) {
        rc = select_plan_nd(p, opts, &choice);
        if (rc != OFFT_SUCCESS) { free_plan(p); set_error(rc); return nullptr; }
    }
    p->ndc = choice;
    p->npass = build_passes_nd(choice, p->nd_dims, batch, p->passes);
    for (int i = 0; i < p->npass && rc == OFFT_SUCCESS; ++i)
        if (!p->passes[i].k) rc = OFFT_ERR_UNSUPPORTED_SIZE;
    if (rc == OFFT_SUCCESS) rc = attach_twiddles(p, p->passes, p->npass, s);
    if (rc == OFFT_SUCCESS && hipStreamSynchronize(s) != hipSuccess) rc = OFFT_ERR_HIP;
    p->use_graph = opts.use_graph;
    if (rc == OFFT_SUCCESS && p->use_graph && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        p->cap = nullptr;
        rc = OFFT_ERR_HIP;
    }
    if (rc != OFFT_SUCCESS) { free_plan(p); set_error(rc); return nullptr; }
    set_error(OFFT_SUCCESS);
    return p;
}

int offt_plan_string_nd(int ndim, const int64_t* dims, int dtype, const char* plan, char* buf, size_t n) {
    int rc = validate_nd(ndim, dims, dtype, 1);
    if (rc == OFFT_SUCCESS && (ndim < 4 || (!buf && n))) rc = OFFT_ERR_INVALID_ARG;
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    NdChoice c = default_choice_nd(dtype, ndim, dims);
    if (plan && !nd_choice_from_string(plan, dtype, ndim, dims, &c, false)) {
        set_error(OFFT_ERR_BAD_PLAN);
        return OFFT_ERR_BAD_PLAN;
    }
    const std::string s = nd_choice_to_string(c, dims);
    if (n) {
        const size_t m = std::min(n - 1, s.size());
        memcpy(buf, s.data(), m);
        buf[m] = 0;
    }
    set_error(OFFT_SUCCESS);
    return (int)s.size();
}

// use_graph: capture the passes for (in, out, dir) on the plan's private
// stream.  Each direction has its own instantiated graph: the first capture
// is instantiated, later ones (other buffers) update it in place
// (re-instantiated only if the update is refused).  The graphs hold only the
// pass kernels.
static int capture_passes(offt_plan_s* p, const void* in, void* out, int dir) {
    const int d = dir > 0 ? 1 : 0;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        return OFFT_ERR_HIP;
    }
    const int rc = exec_passes(p, dir_passes(p, dir), p->npass, in, out, p->work, dir, p->cap);
    const hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (rc != OFFT_SUCCESS || e != hipSuccess || !g) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return OFFT_ERR_HIP;
    }
    bool updated = false;
    if (p->gexec[d]) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        updated = hipGraphExecUpdate(p->gexec[d], g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(p->gexec[d]);
            p->gexec[d] = nullptr;
        }
    }
    if (!updated && hipGraphInstantiate(&p->gexec[d], g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        p->gexec[d] = nullptr;
        (void)hipGraphDestroy(g);
        return OFFT_ERR_HIP;
    }
    if (p->graph[d]) (void)hipGraphDestroy(p->graph[d]);
    p->graph[d] = g;
    p->g_in[d] = in;
    p->g_out[d] = out;
    return OFFT_SUCCESS;
}

// normalize: -1 the plan's normalize_inverse, 0 or 1 this call's choice (the
// graphs hold the plan's scaling, so another choice launches directly)
static int exec_checked(offt_plan_t p, const void* in, void* out, void* stream, int dir, int normalize = -1) {
    if (!p || !in || !out || normalize < -1 || normalize > 1) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    if (p->kind != 1 && p->kind != 3 && p->kind != 4) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = OFFT_SUCCESS;
    if (p->kind == 4) {
        rc = exec_dist(p, dir, 5, in, out, -1, normalize, s);
        set_error(rc);
        return rc;
    }
    if (normalize == p->normalize) normalize = -1;
    if (p->use_graph && p->npass > 0 && normalize < 0) {
        const int d = dir > 0 ? 1 : 0;
        if (!p->gexec[d] || in != p->g_in[d] || out != p->g_out[d]) rc = capture_passes(p, in, out, dir);
        if (rc == OFFT_SUCCESS && hipGraphLaunch(p->gexec[d], s) != hipSuccess) {
            (void)hipGetLastError();
            rc = OFFT_ERR_HIP;
        }
    } else {
        rc = exec_passes(p, dir_passes(p, dir), p->npass, in, out, p->work, dir, s, normalize);
    }
    set_error(rc);
    return rc;
}

int offt_exec_fwd(offt_plan_t p, const void* in, void* out, void* stream) {
    return exec_checked(p, in, out, stream, OFFT_FORWARD);
}

int offt_exec_bwd(offt_plan_t p, const void* in, void* out, void* stream) {
    return exec_checked(p, in, out, stream, OFFT_BACKWARD);
}

int offt_exec_bwd_norm(offt_plan_t p, const void* in, void* out, int normalize, void* stream) {
    return exec_checked(p, in, out, stream, OFFT_BACKWARD, normalize);
}

int offt_plan_passes(offt_plan_t p) {
    if (!p) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    if (p->kind != 1 && p->kind != 3) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    set_error(OFFT_SUCCESS);
    return p->npass;
}

int offt_exec_pass(offt_plan_t p, int i, int direction, const void* in, void* out, void* stream) {
    if (!p || !in || !out || (direction != OFFT_FORWARD && direction != OFFT_BACKWARD)) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    if (p->kind != 1 && p->kind != 3) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    if (i < 0 || i >= p->npass) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    const int rc = exec_passes(p, dir_passes(p, direction), p->npass, in, out, p->work, direction,
                               static_cast<hipStream_t>(stream), -1, i, i + 1);
    set_error(rc);
    return rc;
}

int offt_exec_range(offt_plan_t p, int first, int count, int direction, const void* in, void* out,
                    void* stream) {
    if (!p || !in || !out || (direction != OFFT_FORWARD && direction != OFFT_BACKWARD)) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    if (p->kind != 1 && p->kind != 3) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    if (first < 0 || count < 1 || first > p->npass - count) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    const int rc = exec_passes(p, dir_passes(p, direction), p->npass, in, out, p->work, direction,
                               static_cast<hipStream_t>(stream), -1, first, first + count);
    set_error(rc);
    return rc;
}

int offt_destroy(offt_plan_t p) {
    free_plan(p);
    set_error(OFFT_SUCCESS);
    return OFFT_SUCCESS;
}

int offt_plan_describe(offt_plan_t p, char* buf, size_t n) {
    if (!p || (!buf && n)) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    std::string s = describe_plan(p);
    if (n) {
        const size_t m = std::min(n - 1, s.size());
        memcpy(buf, s.data(), m);
        buf[m] = 0;
    }
    set_error(OFFT_SUCCESS);
    return (int)s.size();
}

int64_t offt_workspace_bytes(offt_plan_t p) {
    if (!p) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    set_error(OFFT_SUCCESS);
    return p->workspace_bytes();
}

int offt_default_plan_string(int64_t Na, int64_t Nb, int64_t Nc, int dtype, char* buf, size_t n) {
    const int rc = validate_dims(Na, Nb, Nc, dtype, 1);
    if (rc != OFFT_SUCCESS || (!buf && n)) {
        const int e = rc != OFFT_SUCCESS ? rc : OFFT_ERR_INVALID_ARG;
        set_error(e);
        return e;
    }
    const int64_t dims[3] = {Na, Nb, Nc};
    const std::string s = choice_to_string(default_choice(dtype, dims), dims);
    if (n) {
        const size_t m = std::min(n - 1, s.size());
        memcpy(buf, s.data(), m);
        buf[m] = 0;
    }
    set_error(OFFT_SUCCESS);
    return (int)s.size();
}

int offt_plan_string(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int layout, const char* plan, char* buf,
                     size_t n) {
    int rc = validate_dims(Na, Nb, Nc, dtype, 1);
    if (rc == OFFT_SUCCESS && ((!buf && n) || (layout != OFFT_LAYOUT_NATURAL && layout != OFFT_LAYOUT_REVERSED)))
        rc = OFFT_ERR_INVALID_ARG;
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    const int64_t dims[3] = {Na, Nb, Nc};
    int64_t rdims[3];
    reversed_dims(dims, rdims);
    const bool reversed = layout == OFFT_LAYOUT_REVERSED;
    const bool moves = reversed && reversal_moves_data(dims);
    PlanChoice c = reversed ? default_choice_reversed(dtype, dims) : default_choice(dtype, dims);
    PlanChoice cb = reversed ? default_choice_reversed(dtype, rdims) : c;
    if (plan) {
        const std::string fp(plan);
        const size_t bar = fp.find('|');
        bool ok = (bar != std::string::npos) == reversed &&
                  choice_from_string(fp.substr(0, bar).c_str(), dtype, dims, &c, false);
        if (ok && reversed) ok = choice_from_string(fp.substr(bar + 1).c_str(), dtype, rdims, &cb, false);
        if (ok) ok = (c.tax >= 0) == moves && (!reversed || (cb.tax >= 0) == moves);
        if (!ok) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    }
    std::string s = choice_to_string(c, dims);
    if (reversed) s += "|" + choice_to_string(cb, rdims);
    if (n) {
        const size_t m = std::min(n - 1, s.size());
        memcpy(buf, s.data(), m);
        buf[m] = 0;
    }
    set_error(OFFT_SUCCESS);
    return (int)s.size();
}

int offt_twiddles(int64_t n, int dtype, void* host_out) {
    if (n < 1 || !host_out || (dtype != OFFT_C2C_F64 && dtype != OFFT_C2C_F32)) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    int rc = check_device();
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    void* d = nullptr;
    const size_t bytes = (size_t)n * elem_size(dtype);
    if (hipMalloc(&d, bytes) != hipSuccess) { set_error(OFFT_ERR_OUT_OF_MEMORY); return OFFT_ERR_OUT_OF_MEMORY; }
    rc = OFFT_SUCCESS;
    if (launch_twiddles(d, n, dtype, nullptr) != hipSuccess ||
        hipMemcpy(host_out, d, bytes, hipMemcpyDeviceToHost) != hipSuccess)
        rc = OFFT_ERR_HIP;
    (void)hipFree(d);
    set_error(rc);
    return rc;
}

}  // extern "C"
