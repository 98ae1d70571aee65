// many_device.hpp -- persistent executor for a batch of grids of different
// sizes.
//
// One launch runs every (grid, axis pass, tile) work item of the batch.  Work
// items are ordered pass level by pass level: all first passes of all grids,
// then all second passes, then all third passes; a "segment" is the run of
// tiles of one (level, grid).  Workgroups pop items from one queue counter in
// increasing order.  An item of level p > 0 may start only when every tile of
// the same grid's level p-1 segment has been published.
//
// Progress: when a workgroup takes item i, every item < i has already been
// taken by a workgroup that is resident and running, and an item depends only
// on items of a lower level, i.e. smaller indices.  So the smallest unfinished
// item never waits, by induction every wait ends, and the number of resident
// workgroups does not matter.  Each wait is still bounded: after spin_limit
// polls the error flag is raised; from then on no wait spins and no item is
// computed, so the grid drains within about one spin limit.
//
// A work item covers tiles_per_item consecutive tiles of one segment, so the
// publish/wait cost is paid once per several tiles.
//
// Visibility across XCDs (each XCD has its own L2): tiles are written with
// agent-scope (write-through) stores, and every thread waits until its
// stores have completed (vmcnt 0) before the workgroup barrier; then one
// thread publishes with an agent-scope release atomic.  Because the executor
// leaves no dirty tile data in any L2, that release's L2 write-back is cheap.
// The consumer polls the counter with relaxed agent-scope loads, then one
// thread performs an agent-scope acquire (L1/L2 invalidate) before the
// workgroup barrier that releases the other threads onto the data.  Tiles of
// a grid's last pass publish nothing (nothing depends on them) and
// first-pass tiles wait for nothing.
#pragma once

#include "fft_device.hpp"

namespace offt {

struct ManySeg {
    int64_t elem_off;    // element offset of the grid in the packed buffer
    int64_t nlines;      // lines of this pass
    int64_t M2;          // element stride of the pass axis
    int64_t item_base;   // first work item of the segment (items, not tiles)
    int64_t tile_base;   // first tile of the segment in the level kernels' tile numbering
    int64_t group_tile_base;   // first tile of the segment within its (level, case) group
    const void* tw;      // twiddle table of the pass length
    double scale_bwd;    // scale of the grid's last pass in a backward transform
    int kid;             // kernel case in the executor's dispatch table
    int logW;            // lines per tile = 2^logW
    int mode;            // 0 contiguous lines, 1 strided lines
    int ntiles;          // tiles of W lines
    int nitems;          // work items = ceil(ntiles / tiles_per_item)
    int first;           // the grid's first pass: reads the input buffer
    int last;            // the grid's last pass
    int dep;             // segment that must complete first, or -1
    int tiles_per_item;  // consecutive tiles one work item covers
};

struct ManyArgs {
    const void* in;
    void* out;
    const ManySeg* segs;
    unsigned* counters;  // [0] queue head, [1] error flag, [2 + s] items done in segment s
    int64_t total_items;
    int nseg;
    int dir;             // -1 forward, +1 backward
    int spin_limit;
    int pad_;
};

constexpr int kManyCounterBase = 2;

// Waits until this thread's outstanding memory operations have completed
// (stores acknowledged by L2).
__device__ __forceinline__ void wait_own_stores() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);   // keep the compiler from moving stores past the wait
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// The tiles of work item `item` of segment `sg`, one after the other.
template <typename V, typename Dispatch>
__device__ __forceinline__ void run_item(const ManySeg& sg, const PassArgs& p, int64_t item, V* __restrict__ lds,
                                         const Dispatch& dispatch) {
    const int64_t t0 = (item - sg.item_base) * sg.tiles_per_item;
    for (int k = 0; k < sg.tiles_per_item; ++k) {
        const int64_t tile = t0 + k;
        if (tile >= sg.ntiles) break;   // uniform across the workgroup
        if (k > 0) __syncthreads();     // the previous tile is done with LDS
        dispatch(sg.kid, p, lds, tile << sg.logW);
    }
}

// Segment of work item `item`: the last segment with item_base <= item.
__device__ __forceinline__ int find_segment(const ManySeg* segs, int nseg, int64_t item) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].item_base <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename V>
__device__ __forceinline__ PassArgs segment_pass_args(const ManyArgs& a, const ManySeg& sg) {
    const bool bwd = a.dir > 0;
    PassArgs p;
    p.in = static_cast<const V*>(sg.first ? a.in : a.out) + sg.elem_off;
    p.out = static_cast<V*>(a.out) + sg.elem_off;
    p.tw = sg.tw;
    p.nlines = sg.nlines;
    p.M2 = sg.M2;
    p.logW = sg.logW;
    p.mode = sg.mode;
    p.X = 1;
    p.Y = 1;
    p.xcd_remap = 0;   // the batch executors map tiles themselves
    p.stream_io = 0;
    p.conj_in = bwd && sg.first;
    p.conj_out = bwd && sg.last;
    p.scale = (bwd && sg.last) ? sg.scale_bwd : 1.0;
    return p;
}

// Error flag of a persistent run (counters[1]): raised by the first wait that
// reaches its spin limit.  Once it is up, no later wait spins: the run's
// results are invalid anyway, so every workgroup drains the queue without
// computing and the kernel ends within about one spin limit.
__device__ __forceinline__ bool many_failed(const ManyArgs& a) {
    return __hip_atomic_load(&a.counters[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

// Polls *counter until it reaches target, the spin limit is hit (raises the
// error flag) or the flag is up.  Returns whether the target was reached.
constexpr int kFlagPollInterval = 64;   // polls between two looks at the error flag
__device__ __forceinline__ bool many_wait(const ManyArgs& a, const unsigned* counter, unsigned target) {
    int polls = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (polls % kFlagPollInterval == 0 && many_failed(a)) return false;
        if (++polls > a.spin_limit) {
            __hip_atomic_store(&a.counters[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(4);
    }
    return true;
}

template <typename V, typename Dispatch>
__device__ __forceinline__ void many_body(const ManyArgs& a, V* __restrict__ lds, const Dispatch& dispatch) {
    __shared__ int64_t s_item;
    __shared__ int s_seg;
    __shared__ int s_run;
    const int tid = threadIdx.x;
    for (;;) {
        __syncthreads();   // the previous tile is done with LDS and the broadcast slots
        if (tid == 0) {
            const int64_t item = (int64_t)__hip_atomic_fetch_add(&a.counters[0], 1u, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
            int seg = -1;
            bool run = false;
            if (item < a.total_items) {
                seg = find_segment(a.segs, a.nseg, item);
                const int dep = a.segs[seg].dep;
                run = !many_failed(a);
                if (run && dep >= 0) {
                    run = many_wait(a, &a.counters[kManyCounterBase + dep], (unsigned)a.segs[dep].nitems);
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
            }
            s_item = item;
            s_seg = seg;
            s_run = run ? 1 : 0;
        }
        __syncthreads();
        const int64_t item = s_item;
        const int seg = s_seg;
        if (item >= a.total_items) break;
        if (!s_run) continue;   // a wait failed: drain the queue without computing
        const ManySeg sg = a.segs[seg];
        const PassArgs p = segment_pass_args<V>(a, sg);
        run_item(sg, p, item, lds, dispatch);
        if (!sg.last) {
            wait_own_stores();
            __syncthreads();
            if (tid == 0)
                __hip_atomic_fetch_add(&a.counters[kManyCounterBase + seg], 1u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Segment of tile `tile` in the level kernels' numbering: the last segment
// with tile_base <= tile.
__device__ __forceinline__ int find_segment_by_tile(const ManySeg* segs, int nseg, int64_t tile) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Non-persistent form: one workgroup per tile of tiles
// [tile_begin, tile_begin + gridDim.x), all of one pass level, so the kernel
// boundary between levels orders the passes and no counters are used.
template <typename V, typename Dispatch>
__device__ __forceinline__ void many_level_body(const ManyArgs& a, int64_t tile_begin, V* __restrict__ lds,
                                                const Dispatch& dispatch) {
    const int64_t tile = tile_begin + (int64_t)blockIdx.x;
    const int seg = find_segment_by_tile(a.segs, a.nseg, tile);
    const ManySeg sg = a.segs[seg];
    const PassArgs p = segment_pass_args<V>(a, sg);
    dispatch(sg.kid, p, lds, (tile - sg.tile_base) << sg.logW);
}

// ---- level-synchronous persistent form ------------------------------------
// One launch of gridDim.x workgroups, all resident.  Pass level by pass
// level the workgroups take the level's tiles from queues, then meet at a
// grid barrier after each level.  A level's tiles are split into kXcds
// ranges, one queue counter each: range x holds, case after case, the x-th
// share of every (level, kernel case) group's tiles (the group's segments in
// grid order), cut into items of kSyncTilesPerPop consecutive tiles of one
// case.  A workgroup pops items from the range of its own XCD (workgroups go
// to the XCDs round-robin in launch order), then from the others'.  Item
// numbers only grow, so a workgroup walks the cases in order, each case's
// items in a loop of its own: the case's code is inlined without a loop
// around a switch over all cases (whose hoisted values would all stay live),
// and a range costs one pop per item plus one that finds it empty.  The next
// item is popped before the current one runs, so the atomic's round trip
// overlaps the tile's loads.  Tiles use plain stores; the barrier makes them
// visible across XCDs: every thread waits for its stores, then one thread
// releases at agent scope (L2 write-back), arrives, waits for all
// workgroups, and acquires (L2 invalidate).  A barrier wait gives up after
// spin_limit polls and raises the error flag, so the grid always drains even
// if not every workgroup is resident (the results are then invalid and
// offt_many_status says so).
constexpr int kSyncTilesPerPop = 4;

struct ManyGroup {
    int seg_begin;       // [seg_begin, seg_end) into ManySyncArgs::gseg
    int seg_end;
    int64_t ntiles;      // tiles of the group
};

// The items of one (level, XCD range, case): items [item_begin, item_end) of
// the range's queue cover the group's tiles [tile_begin, tile_end).
struct ManyRange {
    int64_t item_begin;
    int64_t item_end;
    int64_t tile_begin;
    int64_t tile_end;
};

struct ManySyncArgs {
    const ManyGroup* groups;   // [level * ncases + case]
    const int* gseg;           // segment indices, grouped by (level, case), grid order within a group
    const ManyRange* ranges;   // [(level * kXcds + x) * ncases + case]
    unsigned* queue;           // [level * kXcds + x]: items taken from range x (zeroed)
    unsigned* barrier;         // one arrival counter per level boundary (zeroed before the launch)
    int ncases;
    int pad_;
};

// Items of case kid in range `rg` while the workgroup's current item `*item`
// (the same in every thread) falls in them; pops the next one from `queue`.
template <typename V, typename TileFn>
__device__ __forceinline__ void many_sync_case(const ManyArgs& a, const ManySyncArgs& g, int lvl, int kid,
                                               const ManyRange* rg, unsigned* queue, int64_t* item,
                                               int64_t* s_next, TileFn&& tile) {
    if (kid >= g.ncases) return;   // a table of fewer cases than the kernel's: nothing to run
    const ManyRange r = rg[kid];
    if (*item >= r.item_end) return;
    const ManyGroup gr = g.groups[lvl * g.ncases + kid];
    while (*item < r.item_end) {
        unsigned next = 0;
        if (threadIdx.x == 0)
            next = __hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t t0 = r.tile_begin + (*item - r.item_begin) * kSyncTilesPerPop;
        const int64_t t1 = t0 + kSyncTilesPerPop < r.tile_end ? t0 + kSyncTilesPerPop : r.tile_end;
        for (int64_t t = t0; t < t1; ++t) {
            // segment of group tile t: the last with group_tile_base <= t
            int lo = gr.seg_begin, hi = gr.seg_end - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.segs[g.gseg[mid]].group_tile_base <= t) lo = mid;
                else hi = mid - 1;
            }
            const ManySeg sg = a.segs[g.gseg[lo]];
            const PassArgs p = segment_pass_args<V>(a, sg);
            if (t > t0) __syncthreads();   // the previous tile is done with LDS
            tile(p, (t - sg.group_tile_base) << sg.logW);
        }
        __syncthreads();   // the tiles are done with LDS and every thread has read the broadcast slot
        if (threadIdx.x == 0) *s_next = (int64_t)next;
        __syncthreads();
        *item = *s_next;
    }
}

__device__ __forceinline__ void many_grid_barrier(const ManyArgs& a, unsigned* counter) {
    wait_own_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        (void)many_wait(a, counter, gridDim.x);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Every range of one level, the workgroup's own XCD's first, each range's
// cases in case order.  Case types provide `static constexpr int kid` and
// `static void tile(const PassArgs&, V* lds, int64_t l0)`.
template <typename V, typename... Cases>
__device__ __forceinline__ void many_sync_level(const ManyArgs& a, const ManySyncArgs& g, int lvl, V* __restrict__ lds,
                                                int64_t* s_next) {
    const int own = (int)(blockIdx.x % kXcds);
    for (int v = 0; v < kXcds; ++v) {
        const int x = (own + v) % kXcds;
        const ManyRange* rg = g.ranges + (int64_t)(lvl * kXcds + x) * g.ncases;
        if (g.ncases == 0 || rg[g.ncases - 1].item_end == 0) continue;   // an empty range: no pop
        unsigned* queue = g.queue + lvl * kXcds + x;
        __syncthreads();   // every thread has read the broadcast slot
        if (threadIdx.x == 0)
            *s_next = (int64_t)__hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        int64_t item = *s_next;
        (many_sync_case<V>(a, g, lvl, Cases::kid, rg, queue, &item, s_next,
                           [&](const PassArgs& p, int64_t l0) { Cases::tile(p, lds, l0); }),
         ...);
    }
}

// The whole transform of the batch: three levels, two grid barriers (the
// levels written out, so that no value is kept live from one level's loops
// into the next).
template <typename V, typename... Cases>
__device__ __forceinline__ void many_sync_body(const ManyArgs& a, const ManySyncArgs& g, V* __restrict__ lds) {
    __shared__ int64_t s_next;
    many_sync_level<V, Cases...>(a, g, 0, lds, &s_next);
    many_grid_barrier(a, g.barrier + 0);
    many_sync_level<V, Cases...>(a, g, 1, lds, &s_next);
    many_grid_barrier(a, g.barrier + 1);
    many_sync_level<V, Cases...>(a, g, 2, lds, &s_next);
}

}  // namespace offt
