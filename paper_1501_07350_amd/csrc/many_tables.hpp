// many_tables.hpp -- host-side work-item tables of the uneven-batch
// executors (many.hip): segments (one per grid and pass level), their tile
// widths, tile and work-item numbering, level boundaries and the launch's
// dynamic LDS.  Plain C++ over the device structs of many_device.hpp, so the
// library and the CPU emulation of the executors build the same tables.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "many_device.hpp"

namespace offt {

constexpr int kManyThreads = 512;   // workgroup size of every executor kernel
// LDS per workgroup of the executors: three fit in a CU's 160 KiB (the level
// kernels' 65 registers allow three 512-thread workgroups per CU; on 64
// uneven complex64 grids 52 KiB beat 80 KiB by 16% and 40 KiB by 2%)
constexpr int64_t kManyLdsBudget = 52 * 1024;
constexpr int kTilesPerItem = 4;    // tiles of one work item of the queue-based persistent kernel

// One axis pass of one grid, as the executors see it.
struct ManyPassDesc {
    int L;                // line length
    int64_t nlines;       // lines of the pass (M1 * M2)
    int64_t M2;           // element stride of the axis
    int mode;             // 0 contiguous lines, 1 strided lines
    int tpl;              // threads per line of the kernel case
    int kid;              // kernel case in the executor's dispatch table (-1: none)
    const void* tw;       // twiddle table of L
};

struct ManyGridDesc {
    int64_t elem_off;                   // element offset in the packed buffer
    double scale_bwd;                   // scale of the last pass of a backward transform
    std::vector<ManyPassDesc> passes;   // in pass order
};

struct ManyTables {
    std::vector<ManySeg> segs;          // level-major, grid order within a level
    int64_t level_begin[4] = {0, 0, 0, 0};        // work items of level l: [level_begin[l], level_begin[l+1])
    int64_t level_tile_begin[4] = {0, 0, 0, 0};   // tiles of level l (level kernels, level-synchronous form)
    int64_t total_items = 0;
    size_t lds_bytes = 0;               // dynamic LDS of the launch: the largest tile
    std::vector<int> seg_level;         // pass level of each segment
    std::vector<int> tile_seg;          // [tile]: segment of each tile (level kernels' numbering)
};

// Counters of the level-synchronous form, after the segment counters from a
// 256-byte boundary on: its two level barriers, each alone in 256 bytes.
constexpr int kManySyncCounters = 2 * kManySyncStride;
inline int64_t many_sync_base(int64_t nseg) {
    return (kManyCounterBase + nseg + kManySyncStride - 1) / kManySyncStride * kManySyncStride;
}

// Tile width of a pass inside the executors: as many lines as fill `threads`
// threads, within `lds_budget` bytes of LDS.
inline int many_tile_logW(const ManyPassDesc& p, int64_t elem_bytes, int threads, int64_t lds_budget) {
    int lw = 0;
    while ((int64_t(2) << lw) * p.tpl <= threads && tile_lds_elems(2 << lw, p.L) * elem_bytes <= lds_budget) ++lw;
    return lw;
}

inline void build_many_tables(const std::vector<ManyGridDesc>& grids, int64_t elem_bytes, int threads,
                              int64_t lds_budget, int tiles_per_item, ManyTables* t) {
    const int count = (int)grids.size();
    std::vector<int> seg_of((size_t)count * 3, -1), seg_level;
    t->segs.clear();
    t->lds_bytes = 0;
    for (int lvl = 0; lvl < 3; ++lvl) {
        for (int g = 0; g < count; ++g) {
            const ManyGridDesc& G = grids[g];
            if (lvl >= (int)G.passes.size()) continue;
            const ManyPassDesc& pp = G.passes[lvl];
            ManySeg sg;
            memset(&sg, 0, sizeof sg);
            sg.elem_off = G.elem_off;
            sg.nlines = pp.nlines;
            sg.M2 = pp.M2;
            sg.tw = pp.tw;
            sg.scale_bwd = G.scale_bwd;
            sg.kid = pp.kid;
            sg.logW = many_tile_logW(pp, elem_bytes, threads, lds_budget);
            sg.mode = pp.mode;
            const int64_t W = int64_t(1) << sg.logW;
            sg.ntiles = (int)((sg.nlines + W - 1) / W);
            sg.tiles_per_item = tiles_per_item;
            sg.nitems = (sg.ntiles + tiles_per_item - 1) / tiles_per_item;
            sg.first = lvl == 0;
            sg.last = lvl == (int)G.passes.size() - 1;
            sg.dep = lvl > 0 ? seg_of[(size_t)(lvl - 1) * count + g] : -1;
            seg_of[(size_t)lvl * count + g] = (int)t->segs.size();
            seg_level.push_back(lvl);
            t->lds_bytes = std::max(t->lds_bytes, (size_t)(tile_lds_elems((int)W, pp.L) * elem_bytes));
            t->segs.push_back(sg);
        }
    }
    int64_t items = 0, tiles = 0;
    int lv = 0;
    for (int l = 0; l < 4; ++l) t->level_begin[l] = t->level_tile_begin[l] = 0;
    for (size_t i = 0; i < t->segs.size(); ++i) {
        while (lv < seg_level[i]) {
            ++lv;
            t->level_begin[lv] = items;
            t->level_tile_begin[lv] = tiles;
        }
        t->segs[i].item_base = items;
        t->segs[i].tile_base = tiles;
        items += t->segs[i].nitems;
        tiles += t->segs[i].ntiles;
    }
    while (lv < 3) {
        ++lv;
        t->level_begin[lv] = items;
        t->level_tile_begin[lv] = tiles;
    }
    // segment of every tile of the level kernels' numbering
    t->tile_seg.assign((size_t)tiles, 0);
    for (size_t i = 0; i < t->segs.size(); ++i)
        std::fill(t->tile_seg.begin() + t->segs[i].tile_base,
                  t->tile_seg.begin() + t->segs[i].tile_base + t->segs[i].ntiles, (int)i);
    t->total_items = items;
    t->seg_level = seg_level;
}

// Grouped level schedule: consecutive grids in groups of at most
// `group_bytes` of grid data (a larger grid alone), and per group its three
// pass levels, so that a group's later levels find the earlier ones' output
// in the Infinity Cache.  `map` lists the level kernels' tile numbers group
// by group and level by level; range r = 3 g + l of `ranges` is
// [ranges[r], ranges[r + 1]) of `map`.
struct ManyGroups {
    std::vector<int> map;
    std::vector<int64_t> ranges;   // 3 * groups + 1 entries
    int groups = 0;
};

inline void build_many_groups(const std::vector<ManyGridDesc>& grids, const ManyTables& t, int64_t elem_bytes,
                              int64_t group_bytes, ManyGroups* out) {
    const int count = (int)grids.size();
    // group of every grid, in grid order
    std::vector<int> group_of(count, 0);
    int g = 0;
    int64_t bytes = 0;
    for (int i = 0; i < count; ++i) {
        // the grid's points: its first pass covers them all (lines x length)
        const int64_t n = grids[i].passes.empty() ? 0 : grids[i].passes[0].nlines * grids[i].passes[0].L;
        const int64_t b = n * elem_bytes;
        if (bytes > 0 && bytes + b > group_bytes) {
            ++g;
            bytes = 0;
        }
        group_of[i] = g;
        bytes += b;
    }
    out->groups = count ? g + 1 : 0;
    // segments of each (group, level), in the tables' order (grid order
    // within a level); a segment's grid is found by its element offset
    std::vector<int> seg_grid(t.segs.size(), 0);
    {
        int gi = 0;
        for (size_t s = 0; s < t.segs.size(); ++s) {
            if (s > 0 && t.seg_level[s] != t.seg_level[s - 1]) gi = 0;
            while (gi < count && grids[gi].elem_off != t.segs[s].elem_off) ++gi;
            // every segment belongs to a grid of the list (grid order within
            // a level); a miss would leave the segment out of every group
            seg_grid[s] = gi < count ? gi : -1;
        }
    }
    out->map.clear();
    out->ranges.assign((size_t)3 * out->groups + 1, 0);
    for (int gr = 0; gr < out->groups; ++gr) {
        for (int lvl = 0; lvl < 3; ++lvl) {
            out->ranges[(size_t)3 * gr + lvl] = (int64_t)out->map.size();
            for (size_t s = 0; s < t.segs.size(); ++s) {
                if (t.seg_level[s] != lvl || seg_grid[s] < 0 || group_of[seg_grid[s]] != gr) continue;
                for (int k = 0; k < t.segs[s].ntiles; ++k) out->map.push_back((int)(t.segs[s].tile_base + k));
            }
        }
    }
    out->ranges[(size_t)3 * out->groups] = (int64_t)out->map.size();
}

}  // namespace offt
