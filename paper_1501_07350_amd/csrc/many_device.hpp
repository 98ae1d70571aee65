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
    const int* tile_seg; // [tile]: segment of each tile of the level kernels' numbering
    const int* tile_map; // level kernels: launch position -> tile number (grouped schedule), or null
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
    p.lpm = sg.M2;
    p.blk_ld = 0;
    p.blk_off = 0;
    p.blk_logw = -1;
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

// Non-persistent form: one workgroup per tile of tiles
// [tile_begin, tile_begin + gridDim.x), all of one pass level, so the kernel
// boundary between levels orders the passes and no counters are used.  With
// a tile map (grouped schedule) the launch covers map positions instead,
// the tiles of one level of one group of grids.
template <typename V, typename Dispatch>
__device__ __forceinline__ void many_level_body(const ManyArgs& a, int64_t tile_begin, V* __restrict__ lds,
                                                const Dispatch& dispatch) {
    const int64_t pos = tile_begin + (int64_t)blockIdx.x;
    const int64_t tile = a.tile_map ? (int64_t)a.tile_map[pos] : pos;
    const int seg = a.tile_seg[tile];
    const ManySeg sg = a.segs[seg];
    const PassArgs p = segment_pass_args<V>(a, sg);
    dispatch(sg.kid, p, lds, (tile - sg.tile_base) << sg.logW);
}

// ---- level-synchronous persistent form ------------------------------------
// One launch of gridDim.x workgroups, all resident (sized from the
// occupancy of the kernel, three per CU).  Pass level by pass level each
// workgroup runs the level's tiles blockIdx.x, blockIdx.x + gridDim.x, ...
// of the level kernels' numbering -- the order in which the hardware would
// hand the level kernel's workgroups out -- and the workgroups meet at a grid
// barrier after each level.  No atomics are taken per tile: device-scope
// atomics serialise on their address, and a shared tile queue costs more
// than the imbalance it removes (consecutive tiles come from one segment, so
// a round-robin deal gives every workgroup near-equal work).  The tile code
// is one out-of-line call, so the loop keeps only its own few values live.
// Tiles use plain stores; the barrier makes them visible across XCDs: every
// thread waits for its stores, then one thread releases at agent scope (L2
// write-back), arrives, waits for all workgroups, and acquires (L2
// invalidate).  A barrier wait gives up after spin_limit polls and raises
// the error flag, so the grid always drains even if not every workgroup is
// resident (the results are then invalid and offt_many_status says so).
constexpr int kManySyncStride = 64;   // the two barrier counters 256 bytes apart

struct ManySyncArgs {
    int64_t level_tile_begin[4];   // tiles of level l: [level_tile_begin[l], level_tile_begin[l + 1])
    unsigned* barrier;             // [l * kManySyncStride]: arrivals at level boundary l (zeroed before the launch)
};

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

template <typename V, typename Dispatch>
__device__ __forceinline__ void many_sync_body(const ManyArgs& a, const ManySyncArgs& g, V* __restrict__ lds,
                                               const Dispatch& dispatch) {
    for (int lvl = 0; lvl < 3; ++lvl) {
        for (int64_t t = g.level_tile_begin[lvl] + blockIdx.x; t < g.level_tile_begin[lvl + 1]; t += gridDim.x) {
            const ManySeg sg = a.segs[a.tile_seg[t]];
            const PassArgs p = segment_pass_args<V>(a, sg);
            __syncthreads();   // the previous tile is done with LDS
            dispatch(sg.kid, p, lds, (t - sg.tile_base) << sg.logW);
        }
        if (lvl < 2) many_grid_barrier(a, g.barrier + lvl * kManySyncStride);
    }
}

}  // namespace offt
