// many.hip -- uneven batches: `count` grids of different shapes packed in one
// buffer, transformed by one persistent kernel launch over every (grid, axis
// pass, tile) work item, replayed from a HIP graph.  The per-grid plans come
// from the same heuristic / exhaustive tuning as single-shape plans, the GPU
// counterpart of the paper's run-time auto-tuning (Sec. 3.2.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/offt.h"
#include "many_device.hpp"
#include "many_tables.hpp"
#include "offt_internal.h"
#include "plan_impl.h"
#include "selector.h"

namespace offt {

#include "_gen/many_executors.inc"

static const ManyExecutor* const kExecF64[] = {OFFT_MANY_EXECUTORS_F64};
static const ManyExecutor* const kExecF32[] = {OFFT_MANY_EXECUTORS_F32};

__global__ void many_reset_kernel(unsigned* counters, int n) {
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) counters[i] = 0u;
}

constexpr int kManySpinLimit = 1 << 22;    // polls (~2 s) before a wait gives up and flags an error
// grid data per group of the grouped level schedule: three quarters of the
// 256 MB Infinity Cache (on 64 uneven complex64 grids of 552 MB, groups of
// at most 192 MiB beat 128 and 256 MiB)
constexpr int64_t kManyGroupBytes = int64_t(192) << 20;
constexpr int64_t kAlignBytes = 256;       // every grid starts on a 256-byte boundary

struct ManyGrid {
    int64_t dims[3];
    int64_t off;                 // element offset in the packed buffer
    PlanChoice choice;           // plan used by the persistent executor
    PassPlan tuned[3];           // stand-alone passes of that plan
    int ntuned = 0;
    PassPlan heur[3];            // stand-alone passes of the heuristic plan
    int nheur = 0;
};

struct ManyState {
    int count = 0;
    int64_t total_elems = 0;
    std::vector<ManyGrid> grids;
    bool levels_ok = false;      // every pass has a case in the executor: level kernels
    bool persistent_ok = false;  // ... and the executor has the persistent forms
    const ManyExecutor* exec = nullptr;
    std::string why_not;         // why the persistent forms are unavailable
    std::string why_not_levels;  // why the level kernels are unavailable
    ManySeg* d_segs = nullptr;
    unsigned* d_counters = nullptr;
    int nseg = 0;
    int64_t total_items = 0;
    int nblocks = 0;
    size_t lds = 0;
    const void* kernel = nullptr;
    int64_t level_begin[4] = {0, 0, 0, 0};   // work items of pass level l: [level_begin[l], level_begin[l+1])
    int64_t level_tile_begin[4] = {0, 0, 0, 0};   // tiles of pass level l (level kernels, one per workgroup)
    // graph of the persistent launch: reset node -> persistent node
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraphNode_t node_many = nullptr;
    ManyArgs gargs{};
    bool graph_ready = false;
    int* d_tile_seg = nullptr;   // segment of every tile (level kernels, level-synchronous form)
    // level-synchronous persistent form and its graph
    int sync_nblocks = 0;
    hipGraph_t sgraph = nullptr;
    hipGraphExec_t sgexec = nullptr;
    hipGraphNode_t snode = nullptr;
    ManyArgs sargs{};
    bool sgraph_ready = false;
    // graph of the level launches: level 0 -> level 1 -> level 2
    hipGraph_t lgraph = nullptr;
    hipGraphExec_t lgexec = nullptr;
    hipGraphNode_t lnodes[3] = {nullptr, nullptr, nullptr};
    ManyArgs largs{};
    int64_t lbegin[3] = {0, 0, 0};
    int nlevels = 0;
    bool lgraph_ready = false;
    // grouped level schedule: tile map, ranges (3 per group) and its graph
    ManyGroups groups;
    int* d_tile_map = nullptr;
    hipGraph_t ggraph = nullptr;
    hipGraphExec_t ggexec = nullptr;
    std::vector<hipGraphNode_t> gnodes;
    std::vector<int64_t> gbegin;
    ManyArgs ggargs{};
    bool ggraph_ready = false;
    std::string desc;
};

static int find_case(const ManyExecutor* ex, const KernelEntry* k) {
    for (int i = 0; i < ex->ncases; ++i) {
        const ManyCase& c = ex->cases[i];
        if (c.L != k->L || c.tpl != k->tpl || c.nstages != k->nstages) continue;
        bool eq = true;
        for (int j = 0; j < k->nstages; ++j) eq = eq && c.radices[j] == k->radices[j];
        if (eq) return i;
    }
    return -1;
}

// First executor (compact ones first) with a case for every pass of the batch.
static const ManyExecutor* pick_executor(const ManyState* m, int dtype) {
    const ManyExecutor* const* list = dtype == OFFT_C2C_F64 ? kExecF64 : kExecF32;
    const int n = int((dtype == OFFT_C2C_F64 ? sizeof kExecF64 : sizeof kExecF32) / sizeof(ManyExecutor*));
    for (int e = 0; e < n; ++e) {
        bool all = true;
        for (const ManyGrid& G : m->grids)
            for (int i = 0; i < G.ntuned && all; ++i) all = find_case(list[e], G.tuned[i].k) >= 0;
        if (all) return list[e];
    }
    return nullptr;
}

void release_many(offt_plan_s* p) {
    ManyState* m = p->many;
    if (!m) return;
    if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    if (m->lgexec) (void)hipGraphExecDestroy(m->lgexec);
    if (m->lgraph) (void)hipGraphDestroy(m->lgraph);
    if (m->sgexec) (void)hipGraphExecDestroy(m->sgexec);
    if (m->sgraph) (void)hipGraphDestroy(m->sgraph);
    if (m->ggexec) (void)hipGraphExecDestroy(m->ggexec);
    if (m->ggraph) (void)hipGraphDestroy(m->ggraph);
    delete m;
    p->many = nullptr;
}

std::string describe_many(const offt_plan_s* p) { return p->many ? p->many->desc : std::string(); }

static int dev_alloc(offt_plan_s* p, size_t bytes, void** out) {
    if (hipMalloc(out, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return OFFT_ERR_OUT_OF_MEMORY;
    }
    p->allocs.push_back(*out);
    p->alloc_bytes.push_back(bytes);
    return OFFT_SUCCESS;
}


static int build_many(offt_plan_s* p, hipStream_t s) {
    ManyState* m = p->many;
    const int dtype = p->dtype;
    const size_t es = elem_size(dtype);
    m->exec = pick_executor(m, dtype);
    m->levels_ok = m->exec != nullptr;
    m->persistent_ok = m->exec && m->exec->kernel;
    if (!m->exec) m->why_not_levels = "an axis length above 160";
    if (!m->persistent_ok) m->why_not = "an axis length outside the set {48,60,64,80,96,120,128,150,160}";
    // segments, tiles and work items (many_tables.hpp, shared with the CPU
    // emulation of the executors)
    std::vector<ManyGridDesc> gd(m->count);
    for (int g = 0; g < m->count; ++g) {
        const ManyGrid& G = m->grids[g];
        gd[g].elem_off = G.off;
        gd[g].scale_bwd = p->normalize ? 1.0 / (double)(G.dims[0] * G.dims[1] * G.dims[2]) : 1.0;
        for (int i = 0; i < G.ntuned; ++i) {
            const PassPlan& pp = G.tuned[i];
            gd[g].passes.push_back({pp.L, pp.M1 * pp.M2, pp.M2, pp.mode, pp.k->tpl,
                                    m->exec ? find_case(m->exec, pp.k) : -1, pp.tw});
        }
    }
    ManyTables tab;
    build_many_tables(gd, (int64_t)es, kManyThreads, std::min(kManyLdsBudget, lds_limit()), kTilesPerItem, &tab);
    std::vector<ManySeg>& segs = tab.segs;
    const int64_t items = tab.total_items;
    const size_t lds_max = tab.lds_bytes;
    for (int l = 0; l < 4; ++l) {
        m->level_begin[l] = tab.level_begin[l];
        m->level_tile_begin[l] = tab.level_tile_begin[l];
    }
    m->nseg = (int)segs.size();
    m->total_items = items;
    if (items >= (int64_t(1) << 31)) { m->persistent_ok = false; m->why_not = "too many work items"; }
    // a launch holds at most 2^32 - 1 work-items: tiles of one level
    for (int l = 0; l < 3; ++l)
        if ((tab.level_tile_begin[l + 1] - tab.level_tile_begin[l]) * kManyThreads > int64_t(0xffffffffu)) {
            m->levels_ok = m->persistent_ok = false;
            m->why_not_levels = m->why_not = "too many tiles in one pass level";
        }
    if (m->nseg == 0) return OFFT_SUCCESS;   // all grids 1x1x1: copies only
    void* d = nullptr;
    int rc = dev_alloc(p, sizeof(ManySeg) * segs.size(), &d);
    if (rc) return rc;
    m->d_segs = static_cast<ManySeg*>(d);
    rc = dev_alloc(p, sizeof(int) * std::max<size_t>(tab.tile_seg.size(), 1), &d);
    if (rc) return rc;
    m->d_tile_seg = static_cast<int*>(d);
    if (!tab.tile_seg.empty() && hipMemcpyAsync(m->d_tile_seg, tab.tile_seg.data(), sizeof(int) * tab.tile_seg.size(),
                                                hipMemcpyHostToDevice, s) != hipSuccess)
        return OFFT_ERR_HIP;
    // counters: queue head, error flag, one per segment, then the
    // level-synchronous form's two level barriers
    const size_t ncnt = many_sync_base((int64_t)segs.size()) + kManySyncCounters;
    rc = dev_alloc(p, sizeof(unsigned) * ncnt, &d);
    if (rc) return rc;
    m->d_counters = static_cast<unsigned*>(d);
    if (hipMemcpyAsync(m->d_segs, segs.data(), sizeof(ManySeg) * segs.size(), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemsetAsync(m->d_counters, 0, sizeof(unsigned) * ncnt, s) != hipSuccess)
        return OFFT_ERR_HIP;
    if (!m->levels_ok) return OFFT_SUCCESS;
    // grouped level schedule: the level kernels' tiles group by group
    build_many_groups(gd, tab, (int64_t)es, kManyGroupBytes, &m->groups);
    if (!m->groups.map.empty()) {
        rc = dev_alloc(p, sizeof(int) * m->groups.map.size(), &d);
        if (rc) return rc;
        m->d_tile_map = static_cast<int*>(d);
        if (hipMemcpyAsync(m->d_tile_map, m->groups.map.data(), sizeof(int) * m->groups.map.size(),
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return OFFT_ERR_HIP;
    }
    m->lds = std::max<size_t>(lds_max, 16);
    if (m->lds > 65536 &&
        hipFuncSetAttribute(m->exec->level_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)m->lds) !=
            hipSuccess)
        return OFFT_ERR_HIP;
    if (!m->persistent_ok) return OFFT_SUCCESS;
    // occupancy-sized persistent grid
    m->kernel = m->exec->kernel;
    if (m->lds > 65536 &&
        hipFuncSetAttribute(m->kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)m->lds) != hipSuccess)
        return OFFT_ERR_HIP;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, m->kernel, kManyThreads, m->lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return OFFT_ERR_HIP;
    per_cu = std::max(per_cu, 1);
    m->nblocks = (int)std::min<int64_t>(items, (int64_t)per_cu * cus);
    // the level-synchronous kernel: every workgroup resident (its grid barrier
    // waits for all of them), so exactly what fits the device at once
    if (m->lds > 65536 &&
        hipFuncSetAttribute(many_sync_kernel(m->exec), hipFuncAttributeMaxDynamicSharedMemorySize, (int)m->lds) !=
            hipSuccess)
        return OFFT_ERR_HIP;
    int sync_per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&sync_per_cu, many_sync_kernel(m->exec), kManyThreads, m->lds) !=
        hipSuccess)
        return OFFT_ERR_HIP;
    m->sync_nblocks = std::max(sync_per_cu, 1) * cus;
    return OFFT_SUCCESS;
}

static ManyArgs make_args(const ManyState* m, const void* in, void* out, int dir) {
    ManyArgs a;
    memset(&a, 0, sizeof a);
    a.in = in;
    a.out = out;
    a.segs = m->d_segs;
    a.tile_seg = m->d_tile_seg;
    a.counters = m->d_counters;
    a.total_items = m->total_items;
    a.nseg = m->nseg;
    a.dir = dir;
    a.spin_limit = kManySpinLimit;
    return a;
}

static int launch_levels(ManyState* m, const void* in, void* out, int dir, hipStream_t s) {
    ManyArgs a = make_args(m, in, out, dir);
    for (int l = 0; l < 3; ++l) {
        int64_t begin = m->level_tile_begin[l];
        const int64_t n = m->level_tile_begin[l + 1] - begin;
        if (n <= 0) continue;
        void* params[] = {&a, &begin};
        if (hipLaunchKernel(m->exec->level_kernel, dim3((unsigned)n), dim3(kManyThreads), params, m->lds, s) !=
            hipSuccess)
            return OFFT_ERR_HIP;
    }
    return OFFT_SUCCESS;
}

// Graph of the non-empty pass levels, chained; later calls with other buffers
// or direction update the nodes' arguments.
static int level_graph_launch(ManyState* m, const void* in, void* out, int dir, hipStream_t s) {
    ManyArgs a = make_args(m, in, out, dir);
    auto node_params = [&](int l, hipKernelNodeParams* kp, void** params) {
        memset(kp, 0, sizeof *kp);
        params[0] = &m->largs;
        params[1] = &m->lbegin[l];
        kp->func = const_cast<void*>(m->exec->level_kernel);
        kp->gridDim = dim3((unsigned)(m->level_tile_begin[l + 1] - m->level_tile_begin[l]));
        kp->blockDim = dim3(kManyThreads);
        kp->sharedMemBytes = (unsigned)m->lds;
        kp->kernelParams = params;
    };
    if (!m->lgraph_ready) {
        if (hipGraphCreate(&m->lgraph, 0) != hipSuccess) return OFFT_ERR_HIP;
        m->largs = a;
        hipGraphNode_t prev = nullptr;
        for (int l = 0; l < 3; ++l) {
            m->lbegin[l] = m->level_tile_begin[l];
            m->lnodes[l] = nullptr;
            if (m->level_tile_begin[l + 1] <= m->level_tile_begin[l]) continue;
            hipKernelNodeParams kp;
            void* params[2];
            node_params(l, &kp, params);
            if (hipGraphAddKernelNode(&m->lnodes[l], m->lgraph, prev ? &prev : nullptr, prev ? 1 : 0, &kp) !=
                hipSuccess)
                return OFFT_ERR_HIP;
            prev = m->lnodes[l];
        }
        if (hipGraphInstantiate(&m->lgexec, m->lgraph, nullptr, nullptr, 0) != hipSuccess) return OFFT_ERR_HIP;
        m->lgraph_ready = true;
    } else if (memcmp(&a, &m->largs, sizeof a) != 0) {
        m->largs = a;
        for (int l = 0; l < 3; ++l) {
            if (!m->lnodes[l]) continue;
            hipKernelNodeParams kp;
            void* params[2];
            node_params(l, &kp, params);
            if (hipGraphExecKernelNodeSetParams(m->lgexec, m->lnodes[l], &kp) != hipSuccess) return OFFT_ERR_HIP;
        }
    }
    if (hipGraphLaunch(m->lgexec, s) != hipSuccess) return OFFT_ERR_HIP;
    return OFFT_SUCCESS;
}

// Graph of the grouped level schedule: for each group of grids its non-empty
// levels, all chained (one group's levels before the next group's); later
// calls with other buffers or direction update the nodes' arguments.
static int grouped_graph_launch(ManyState* m, const void* in, void* out, int dir, hipStream_t s) {
    ManyArgs a = make_args(m, in, out, dir);
    a.tile_map = m->d_tile_map;
    const int nr = 3 * m->groups.groups;
    auto node_params = [&](int r, hipKernelNodeParams* kp, void** params) {
        memset(kp, 0, sizeof *kp);
        params[0] = &m->ggargs;
        params[1] = &m->gbegin[r];
        kp->func = const_cast<void*>(m->exec->level_kernel);
        kp->gridDim = dim3((unsigned)(m->groups.ranges[r + 1] - m->groups.ranges[r]));
        kp->blockDim = dim3(kManyThreads);
        kp->sharedMemBytes = (unsigned)m->lds;
        kp->kernelParams = params;
    };
    if (!m->ggraph_ready) {
        if (hipGraphCreate(&m->ggraph, 0) != hipSuccess) return OFFT_ERR_HIP;
        m->ggargs = a;
        m->gbegin.assign((size_t)nr, 0);
        m->gnodes.assign((size_t)nr, nullptr);
        hipGraphNode_t prev = nullptr;
        for (int r = 0; r < nr; ++r) {
            m->gbegin[r] = m->groups.ranges[r];
            if (m->groups.ranges[r + 1] <= m->groups.ranges[r]) continue;
            hipKernelNodeParams kp;
            void* params[2];
            node_params(r, &kp, params);
            if (hipGraphAddKernelNode(&m->gnodes[r], m->ggraph, prev ? &prev : nullptr, prev ? 1 : 0, &kp) !=
                hipSuccess)
                return OFFT_ERR_HIP;
            prev = m->gnodes[r];
        }
        if (hipGraphInstantiate(&m->ggexec, m->ggraph, nullptr, nullptr, 0) != hipSuccess) return OFFT_ERR_HIP;
        m->ggraph_ready = true;
    } else if (memcmp(&a, &m->ggargs, sizeof a) != 0) {
        m->ggargs = a;
        for (int r = 0; r < nr; ++r) {
            if (!m->gnodes[r]) continue;
            hipKernelNodeParams kp;
            void* params[2];
            node_params(r, &kp, params);
            if (hipGraphExecKernelNodeSetParams(m->ggexec, m->gnodes[r], &kp) != hipSuccess) return OFFT_ERR_HIP;
        }
    }
    if (hipGraphLaunch(m->ggexec, s) != hipSuccess) return OFFT_ERR_HIP;
    return OFFT_SUCCESS;
}

static int launch_persistent(ManyState* m, const void* in, void* out, int dir, hipStream_t s) {
    const int ncnt = kManyCounterBase + m->nseg;
    hipLaunchKernelGGL(many_reset_kernel, dim3(1), dim3(256), 0, s, m->d_counters, ncnt);
    if (hipGetLastError() != hipSuccess) return OFFT_ERR_HIP;
    ManyArgs a = make_args(m, in, out, dir);
    void* params[] = {&a};
    if (hipLaunchKernel(m->kernel, dim3(m->nblocks), dim3(kManyThreads), params, m->lds, s) != hipSuccess)
        return OFFT_ERR_HIP;
    return OFFT_SUCCESS;
}

static ManySyncArgs make_sync_args(const ManyState* m) {
    ManySyncArgs g;
    memset(&g, 0, sizeof g);
    for (int l = 0; l < 4; ++l) g.level_tile_begin[l] = m->level_tile_begin[l];
    g.barrier = m->d_counters + many_sync_base(m->nseg);
    return g;
}

static int launch_sync(ManyState* m, const void* in, void* out, int dir, hipStream_t s) {
    const int ncnt = (int)(many_sync_base(m->nseg) + kManySyncCounters);
    hipLaunchKernelGGL(many_reset_kernel, dim3(1), dim3(256), 0, s, m->d_counters, ncnt);
    if (hipGetLastError() != hipSuccess) return OFFT_ERR_HIP;
    ManyArgs a = make_args(m, in, out, dir);
    ManySyncArgs g = make_sync_args(m);
    void* params[] = {&a, &g};
    if (hipLaunchKernel(many_sync_kernel(m->exec), dim3(m->sync_nblocks), dim3(kManyThreads), params, m->lds, s) !=
        hipSuccess)
        return OFFT_ERR_HIP;
    return OFFT_SUCCESS;
}

// Graph of the level-synchronous form: counter reset -> persistent kernel.
static int sync_graph_launch(ManyState* m, const void* in, void* out, int dir, hipStream_t s) {
    ManyArgs a = make_args(m, in, out, dir);
    ManySyncArgs g = make_sync_args(m);   // node arguments are copied when the node is set
    auto kernel_params = [&](hipKernelNodeParams* kp, void** params) {
        memset(kp, 0, sizeof *kp);
        params[0] = &m->sargs;
        params[1] = &g;
        kp->func = const_cast<void*>(many_sync_kernel(m->exec));
        kp->gridDim = dim3(m->sync_nblocks);
        kp->blockDim = dim3(kManyThreads);
        kp->sharedMemBytes = (unsigned)m->lds;
        kp->kernelParams = params;
    };
    if (!m->sgraph_ready) {
        if (hipGraphCreate(&m->sgraph, 0) != hipSuccess) return OFFT_ERR_HIP;
        int ncnt = (int)(many_sync_base(m->nseg) + kManySyncCounters);
        unsigned* cnt = m->d_counters;
        void* rparams[] = {&cnt, &ncnt};
        hipKernelNodeParams rp;
        memset(&rp, 0, sizeof rp);
        rp.func = reinterpret_cast<void*>(&many_reset_kernel);
        rp.gridDim = dim3(1);
        rp.blockDim = dim3(256);
        rp.sharedMemBytes = 0;
        rp.kernelParams = rparams;
        hipGraphNode_t reset_node;
        if (hipGraphAddKernelNode(&reset_node, m->sgraph, nullptr, 0, &rp) != hipSuccess) return OFFT_ERR_HIP;
        m->sargs = a;
        hipKernelNodeParams kp;
        void* params[2];
        kernel_params(&kp, params);
        if (hipGraphAddKernelNode(&m->snode, m->sgraph, &reset_node, 1, &kp) != hipSuccess) return OFFT_ERR_HIP;
        if (hipGraphInstantiate(&m->sgexec, m->sgraph, nullptr, nullptr, 0) != hipSuccess) return OFFT_ERR_HIP;
        m->sgraph_ready = true;
    } else if (memcmp(&a, &m->sargs, sizeof a) != 0) {
        m->sargs = a;
        hipKernelNodeParams kp;
        void* params[2];
        kernel_params(&kp, params);
        if (hipGraphExecKernelNodeSetParams(m->sgexec, m->snode, &kp) != hipSuccess) return OFFT_ERR_HIP;
    }
    if (hipGraphLaunch(m->sgexec, s) != hipSuccess) return OFFT_ERR_HIP;
    return OFFT_SUCCESS;
}

// Graph of two kernel nodes (counter reset -> persistent kernel), built once;
// later calls with other buffers or direction update the persistent node's
// arguments in the instantiated graph.
static int graph_launch(ManyState* m, const void* in, void* out, int dir, hipStream_t s) {
    ManyArgs a = make_args(m, in, out, dir);
    if (!m->graph_ready) {
        if (hipGraphCreate(&m->graph, 0) != hipSuccess) return OFFT_ERR_HIP;
        int ncnt = kManyCounterBase + m->nseg;
        unsigned* cnt = m->d_counters;
        void* rparams[] = {&cnt, &ncnt};
        hipKernelNodeParams rp;
        memset(&rp, 0, sizeof rp);
        rp.func = reinterpret_cast<void*>(&many_reset_kernel);
        rp.gridDim = dim3(1);
        rp.blockDim = dim3(256);
        rp.sharedMemBytes = 0;
        rp.kernelParams = rparams;
        hipGraphNode_t reset_node;
        if (hipGraphAddKernelNode(&reset_node, m->graph, nullptr, 0, &rp) != hipSuccess) return OFFT_ERR_HIP;
        m->gargs = a;
        void* mparams[] = {&m->gargs};
        hipKernelNodeParams mp;
        memset(&mp, 0, sizeof mp);
        mp.func = const_cast<void*>(m->kernel);
        mp.gridDim = dim3(m->nblocks);
        mp.blockDim = dim3(kManyThreads);
        mp.sharedMemBytes = (unsigned)m->lds;
        mp.kernelParams = mparams;
        if (hipGraphAddKernelNode(&m->node_many, m->graph, &reset_node, 1, &mp) != hipSuccess) return OFFT_ERR_HIP;
        if (hipGraphInstantiate(&m->gexec, m->graph, nullptr, nullptr, 0) != hipSuccess) return OFFT_ERR_HIP;
        m->graph_ready = true;
    } else if (memcmp(&a, &m->gargs, sizeof a) != 0) {
        m->gargs = a;
        void* mparams[] = {&m->gargs};
        hipKernelNodeParams mp;
        memset(&mp, 0, sizeof mp);
        mp.func = const_cast<void*>(m->kernel);
        mp.gridDim = dim3(m->nblocks);
        mp.blockDim = dim3(kManyThreads);
        mp.sharedMemBytes = (unsigned)m->lds;
        mp.kernelParams = mparams;
        if (hipGraphExecKernelNodeSetParams(m->gexec, m->node_many, &mp) != hipSuccess) return OFFT_ERR_HIP;
    }
    if (hipGraphLaunch(m->gexec, s) != hipSuccess) return OFFT_ERR_HIP;
    return OFFT_SUCCESS;
}

// Per-grid plans for an uneven batch: one choice per distinct shape.
static int choose_many(offt_plan_s* p, const offt_opts& o) {
    ManyState* m = p->many;
    std::map<std::tuple<int64_t, int64_t, int64_t>, PlanChoice> chosen;
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    for (ManyGrid& G : m->grids) {
        const auto key = std::make_tuple(G.dims[0], G.dims[1], G.dims[2]);
        auto it = chosen.find(key);
        if (it == chosen.end()) {
            PlanChoice c = default_choice(p->dtype, G.dims);
            if (o.tune == OFFT_TUNE_EXHAUSTIVE || o.tune == OFFT_TUNE_LEARNED) {
                // tune the shape as a single-grid plan
                offt_plan_s tmp;
                tmp.kind = 1;
                tmp.dtype = p->dtype;
                memcpy(tmp.dims, G.dims, sizeof G.dims);
                tmp.batch = 1;
                offt_opts o2 = o;
                const int rc = select_plan(&tmp, o2, &c, nullptr);
                for (void* d : tmp.allocs) (void)hipFree(d);
                if (rc != OFFT_SUCCESS) return rc;
            }
            it = chosen.emplace(key, c).first;
        }
        G.choice = it->second;
        G.ntuned = build_passes(G.choice, G.dims, 1, G.tuned);
        G.nheur = build_passes(default_choice(p->dtype, G.dims), G.dims, 1, G.heur);
        int rc = attach_twiddles(p, G.tuned, G.ntuned, s);
        if (rc == OFFT_SUCCESS) rc = attach_twiddles(p, G.heur, G.nheur, s);
        if (rc != OFFT_SUCCESS) return rc;
        for (int i = 0; i < G.ntuned; ++i)
            if (!G.tuned[i].k) return OFFT_ERR_UNSUPPORTED_SIZE;
    }
    return OFFT_SUCCESS;
}

static int exec_separate(const offt_plan_s* p, const void* in, void* out, int dir, bool tuned, hipStream_t s) {
    const ManyState* m = p->many;
    const size_t es = elem_size(p->dtype);
    for (const ManyGrid& G : m->grids) {
        offt_plan_s view;   // a single-grid view for exec_passes (no ownership)
        view.kind = 1;
        view.dtype = p->dtype;
        memcpy(view.dims, G.dims, sizeof G.dims);
        view.batch = 1;
        view.normalize = p->normalize;
        const char* gi = static_cast<const char*>(in) + G.off * es;
        char* go = static_cast<char*>(out) + G.off * es;
        const int rc = tuned ? exec_passes(&view, G.tuned, G.ntuned, gi, go, nullptr, dir, s)
                             : exec_passes(&view, G.heur, G.nheur, gi, go, nullptr, dir, s);
        if (rc != OFFT_SUCCESS) return rc;
    }
    return OFFT_SUCCESS;
}

}  // namespace offt

using namespace offt;

extern "C" {

offt_plan_t offt_plan_many(int count, const int64_t* dims, int dtype, const offt_opts* o) {
    offt_opts opts;
    offt_opts_default(&opts);
    if (o) opts = *o;
    if (count < 1 || !dims || (dtype != OFFT_C2C_F64 && dtype != OFFT_C2C_F32) ||
        opts.tune < OFFT_TUNE_NONE || opts.tune > OFFT_TUNE_LEARNED || opts.reps < 1 ||
        opts.layout != OFFT_LAYOUT_NATURAL) {
        set_error(OFFT_ERR_INVALID_ARG);
        return nullptr;
    }
    for (int i = 0; i < count; ++i) {
        const int rc = validate_dims(dims[3 * i], dims[3 * i + 1], dims[3 * i + 2], dtype, 1);
        if (rc != OFFT_SUCCESS) { set_error(rc); return nullptr; }
    }
    int rc = check_device();
    if (rc != OFFT_SUCCESS) { set_error(rc); return nullptr; }
    offt_plan_s* p = new offt_plan_s();
    p->kind = 2;
    p->dtype = dtype;
    p->normalize = opts.normalize_inverse ? 1 : 0;
    p->many = new ManyState();
    ManyState* m = p->many;
    m->count = count;
    m->grids.resize(count);
    const int64_t align = kAlignBytes / (int64_t)elem_size(dtype);
    int64_t off = 0;
    for (int i = 0; i < count; ++i) {
        ManyGrid& G = m->grids[i];
        for (int k = 0; k < 3; ++k) G.dims[k] = dims[3 * i + k];
        G.off = off;
        off += G.dims[0] * G.dims[1] * G.dims[2];
        off = (off + align - 1) / align * align;
    }
    m->total_elems = off;
    hipStream_t s = static_cast<hipStream_t>(opts.stream);
    rc = choose_many(p, opts);
    if (rc == OFFT_SUCCESS) rc = build_many(p, s);
    if (rc == OFFT_SUCCESS && hipStreamSynchronize(s) != hipSuccess) rc = OFFT_ERR_HIP;
    if (rc != OFFT_SUCCESS) { free_plan(p); set_error(rc); return nullptr; }
    char buf[512];
    snprintf(buf, sizeof buf, "many: %d grids, %lld elements, %d segments, %lld work items, executor %s, %d workgroups x %d (level-synchronous: %d), lds %zu, %d level groups%s%s%s%s",
             count, (long long)m->total_elems, m->nseg, (long long)m->total_items, m->exec ? m->exec->name : "-",
             m->nblocks, kManyThreads, m->sync_nblocks, m->lds, m->groups.groups,
             m->levels_ok ? "" : "; level kernels unavailable: ", m->levels_ok ? "" : m->why_not_levels.c_str(),
             m->persistent_ok ? "" : "; persistent executor unavailable: ", m->persistent_ok ? "" : m->why_not.c_str());
    m->desc = buf;
    for (const ManyGrid& G : m->grids) m->desc += "\n" + choice_to_string(G.choice, G.dims);
    set_error(OFFT_SUCCESS);
    return p;
}

int64_t offt_many_offset(offt_plan_t p, int i) {
    if (!p) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    if (p->kind != 2 || !p->many) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    const ManyState* m = p->many;
    if (i < 0 || i > m->count) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    set_error(OFFT_SUCCESS);
    return i == m->count ? m->total_elems : m->grids[i].off;
}

// The default launch of a many-plan: the level kernels replayed from a
// graph (with the grouped schedule, the fastest forms measured on MI355X)
// when an executor covers every pass (every axis at most 160 long), else the
// tuned plans as separate launches.
static int many_default_form(offt_plan_t p) {
    if (!p || p->kind != 2 || !p->many) return OFFT_MANY_LEVELS_GRAPH;   // rejected below
    return p->many->levels_ok ? OFFT_MANY_LEVELS_GRAPH : OFFT_MANY_SEPARATE_TUNED;
}

int offt_exec_many_fwd(offt_plan_t p, const void* in, void* out, void* stream) {
    return offt_exec_many(p, in, out, OFFT_FORWARD, many_default_form(p), stream);
}

int offt_exec_many_bwd(offt_plan_t p, const void* in, void* out, void* stream) {
    return offt_exec_many(p, in, out, OFFT_BACKWARD, many_default_form(p), stream);
}

int offt_exec_many(offt_plan_t p, const void* in, void* out, int direction, int use_graph, void* stream) {
    if (!p || !in || !out || (direction != OFFT_FORWARD && direction != OFFT_BACKWARD) || use_graph < -2 ||
        use_graph > OFFT_MANY_LEVELS_GROUPED_GRAPH) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    if (p->kind != 2 || !p->many) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    ManyState* m = p->many;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = OFFT_SUCCESS;
    if (use_graph >= 0 && in != out) {
        // grids of one point have no pass: copy them
        const size_t es = elem_size(p->dtype);
        for (const ManyGrid& G : m->grids)
            if (G.ntuned == 0 && hipMemcpyAsync(static_cast<char*>(out) + G.off * es,
                                                static_cast<const char*>(in) + G.off * es, es,
                                                hipMemcpyDeviceToDevice, s) != hipSuccess)
                rc = OFFT_ERR_HIP;
    }
    if (rc != OFFT_SUCCESS) {
    } else if (use_graph < 0 || m->nseg == 0) {
        rc = exec_separate(p, in, out, direction, use_graph == -2 || m->nseg == 0, s);
    } else if (use_graph == OFFT_MANY_LEVELS_GRAPH || use_graph == OFFT_MANY_LEVELS ||
               use_graph == OFFT_MANY_LEVELS_GROUPED_GRAPH) {
        if (!m->levels_ok)
            rc = OFFT_ERR_UNSUPPORTED_SIZE;
        else if (use_graph == OFFT_MANY_LEVELS_GRAPH)
            rc = level_graph_launch(m, in, out, direction, s);
        else if (use_graph == OFFT_MANY_LEVELS_GROUPED_GRAPH)
            rc = grouped_graph_launch(m, in, out, direction, s);
        else
            rc = launch_levels(m, in, out, direction, s);
    } else if (!m->persistent_ok) {
        rc = OFFT_ERR_UNSUPPORTED_SIZE;
    } else if (use_graph == OFFT_MANY_PERSISTENT_GRAPH) {
        rc = graph_launch(m, in, out, direction, s);
    } else if (use_graph == OFFT_MANY_PERSISTENT) {
        rc = launch_persistent(m, in, out, direction, s);
    } else if (use_graph == OFFT_MANY_SYNC_GRAPH) {
        rc = sync_graph_launch(m, in, out, direction, s);
    } else {
        rc = launch_sync(m, in, out, direction, s);
    }
    set_error(rc);
    return rc;
}

int offt_many_status(offt_plan_t p) {
    if (!p) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    if (p->kind != 2 || !p->many) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    const ManyState* m = p->many;
    if (!m->d_counters) { set_error(OFFT_SUCCESS); return OFFT_SUCCESS; }
    unsigned flag = 0;
    if (hipMemcpy(&flag, m->d_counters + 1, sizeof flag, hipMemcpyDeviceToHost) != hipSuccess) {
        set_error(OFFT_ERR_HIP);
        return OFFT_ERR_HIP;
    }
    const int rc = flag ? OFFT_ERR_HIP : OFFT_SUCCESS;
    set_error(rc);
    return rc;
}

}  // extern "C"
