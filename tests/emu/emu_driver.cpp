// emu_driver.cpp -- runs the library's tile code (pass_tile) and the
// persistent batch loop (many_body) for one workgroup on CPU threads.
//
//   emu_driver pass <dtype 0|1> <kid> <L> <M1> <M2> <logW> <logP> <TPL>
//       one stand-alone axis pass (kernel case kid of the executor's table,
//       plain stores) over a [M1][L][M2] view of synthetic data, tile by tile
//       with W*TPL threads each (strided lines with LDS exchanges in 2^logP
//       parts when M2 > 1); prints the forward-transformed data as text.
//       EMU_BLK="logw ld off" restricts a strided pass to one column block.
//   emu_driver many <dtype> <nwg> <ngrids> <grids...> <total> [<seg> <dep>]
//       the persistent loop over the segment table the library builds
//       (many_tables.hpp) for the grids' passes, run by nwg workgroups at
//       once: each workgroup is a forked process of kManyThreads CPU
//       threads with exactly the launch's dynamic LDS; buffers and counters
//       live in shared memory.  Each grid: <elem_off> <npass>, then per pass
//       <L> <kid> <mode> <nlines> <M2> <tpl>.  The optional <seg> <dep>
//       makes segment seg wait for segment dep instead.
//   emu_driver sync <dtype> <nwg> <ngrids> <grids...> <total>
//       the level-synchronous persistent body (each level's tiles dealt
//       round-robin, grid barriers between levels) over the batch
//       executor's cases
//   emu_driver tables <dtype> <nwg> <ngrids> <grids...> <total>
//       prints the segment, tile and level tables the library builds for the
//       grids (many_tables.hpp), without running anything
//   emu_driver levels <dtype> <nwg> <ngrids> <grids...> <total>
//       the level kernels' body, one workgroup per tile, level after level,
//       over the batch executor's cases (levels_all: the every-length
//       executor's)
//   emu_driver route <Na> <Nb> <Nc> <np> <in_order> <out_order> <per_chunk>
//       one exchange of the distributed flow with the library's own tables
//       (dist_tables.hpp) and exchange code (dist_device.hpp): every
//       element of the O_in array holds its own O_in index; pack, chunk
//       copies, unpack (per_chunk: one unpack per (src, dst) chunk); prints
//       the chunk counts and the O_out array
//
// Built by tests/test_emu.py with g++ -fsanitize=address.
#include "hip_emu.h"

#include <sys/mman.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "fft_device.hpp"
#include "many_device.hpp"
#include "many_tables.hpp"
#include "dist_device.hpp"
#include "dist_tables.hpp"
#include "emu_cases.inc"

thread_local EmuDim threadIdx;
EmuDim blockIdx, blockDim, gridDim;
EmuBarrier g_emu_barrier;
thread_local long g_emu_barrier_count = 0;

using namespace offt;

template <typename V> static void twiddles(std::vector<V>& tw, int L) {
    tw.resize(L);
    for (int m = 0; m < L; ++m) {
        const double a = 2.0 * M_PI * (double)m / (double)L;
        tw[m].x = (decltype(tw[m].x))std::cos(a);
        tw[m].y = (decltype(tw[m].y))(-std::sin(a));
    }
}

// Runs fn(tid) on `threads` CPU threads that share one barrier; returns false
// if the threads passed different numbers of barriers or a barrier broke.
static bool run_block(int threads, const std::function<void(int)>& fn) {
    g_emu_barrier.reset(threads);
    std::vector<long> counts(threads);
    std::vector<std::thread> ts;
    for (int t = 0; t < threads; ++t)
        ts.emplace_back([&, t] {
            threadIdx.x = (unsigned)t;
            g_emu_barrier_count = 0;
            fn(t);
            counts[t] = g_emu_barrier_count;
        });
    for (auto& th : ts) th.join();
    bool ok = !g_emu_barrier.broken;
    for (int t = 1; t < threads; ++t)
        if (counts[t] != counts[0]) ok = false;
    if (!ok) std::fprintf(stderr, "EMU: barrier counts differ (thread 0: %ld)\n", counts[0]);
    return ok;
}

template <typename V>
static int do_many(int argc, char** argv, bool sync, bool levels = false, bool tables_only = false,
                   bool all_cases = false) {
    int k = 3;
    const int nwg = atoi(argv[k++]);
    const int ngrids = atoi(argv[k++]);
    std::vector<ManyGridDesc> gd(ngrids);
    std::vector<std::vector<V>> tws;
    tws.reserve(64);
    for (int g = 0; g < ngrids; ++g) {
        gd[g].elem_off = atoll(argv[k++]);
        gd[g].scale_bwd = 1.0;
        const int npass = atoi(argv[k++]);
        for (int i = 0; i < npass; ++i) {
            ManyPassDesc d;
            d.L = atoi(argv[k++]);
            d.kid = atoi(argv[k++]);
            d.mode = atoi(argv[k++]);
            d.nlines = atoll(argv[k++]);
            d.M2 = atoll(argv[k++]);
            d.tpl = atoi(argv[k++]);
            tws.emplace_back();
            twiddles(tws.back(), d.L);
            d.tw = nullptr;
            gd[g].passes.push_back(d);
        }
    }
    const int64_t total = atoll(argv[k++]);
    // the library's own tables and launch LDS (no slack: AddressSanitizer
    // flags any access beyond what the GPU launch gets)
    ManyTables tab;
    build_many_tables(gd, (int64_t)sizeof(V), kManyThreads, kManyLdsBudget, kTilesPerItem, &tab);
    std::vector<ManySeg>& segs = tab.segs;
    const int nseg = (int)segs.size();
    if (tables_only) {
        // the tables as the library builds them, one segment per line
        std::printf("TABLES %d segments %lld items %lld tiles lds %zu threads %d tiles_per_item %d\n", nseg,
                    (long long)tab.total_items, (long long)tab.level_tile_begin[3], tab.lds_bytes, kManyThreads,
                    kTilesPerItem);
        for (int i = 0; i < nseg; ++i) {
            const ManySeg& sg = segs[i];
            std::printf("%d %d %lld %lld %lld %d %d %d %d %d %d %d %d %lld %lld\n", i, tab.seg_level[i],
                        (long long)sg.elem_off, (long long)sg.nlines, (long long)sg.M2, sg.kid, sg.logW, sg.mode,
                        sg.ntiles, sg.nitems, sg.first, sg.last, sg.dep, (long long)sg.item_base,
                        (long long)sg.tile_base);
        }
        for (int l = 0; l < 4; ++l) std::printf("level %d %lld %lld\n", l, (long long)tab.level_begin[l],
                                                 (long long)tab.level_tile_begin[l]);
        return 0;
    }
    {
        // twiddle tables: segments follow the level-major order of the table
        std::vector<const void*> tw_of;
        size_t t = 0;
        std::vector<std::vector<const void*>> per_grid(ngrids);
        for (int g = 0; g < ngrids; ++g)
            for (size_t i = 0; i < gd[g].passes.size(); ++i) per_grid[g].push_back(tws[t++].data());
        int s2 = 0;
        for (int lvl = 0; lvl < 3; ++lvl)
            for (int g = 0; g < ngrids; ++g)
                if (lvl < (int)gd[g].passes.size()) segs[s2++].tw = per_grid[g][lvl];
    }
    int64_t waiting_items = 0;
    if (k + 1 < argc) {   // a dependency made unmet on purpose
        const int sgi = atoi(argv[k]);
        if (sgi < 0 || sgi >= (int)segs.size()) return 2;
        segs[sgi].dep = atoi(argv[k + 1]);
        waiting_items = tab.total_items - segs[sgi].item_base;
    }
    const size_t lds_elems = tab.lds_bytes / sizeof(V);
    const int64_t items = tab.total_items;
    const int threads = kManyThreads;
    // shared between the workgroup processes: buffers, counters, two level
    // barriers of the level-synchronous form
    const int ncnt = (int)(many_sync_base(nseg) + kManySyncCounters);
    const size_t bytes = sizeof(V) * 2 * (size_t)total + sizeof(unsigned) * ncnt;
    void* shm = mmap(nullptr, bytes, PROT_READ | PROT_WRITE, MAP_SHARED | MAP_ANONYMOUS, -1, 0);
    if (shm == MAP_FAILED) return 3;
    V* in = static_cast<V*>(shm);
    V* out = in + total;
    unsigned* counters = reinterpret_cast<unsigned*>(out + total);
    for (int64_t i = 0; i < total; ++i) {
        in[i].x = (decltype(in[i].x))std::sin(0.37 * (double)i + 0.1);
        in[i].y = (decltype(in[i].y))std::cos(0.91 * (double)i);
        out[i].x = out[i].y = 0;
    }
    for (int i = 0; i < ncnt; ++i) counters[i] = 0u;
    ManySyncArgs sa;
    memset(&sa, 0, sizeof sa);
    for (int l = 0; l < 4; ++l) sa.level_tile_begin[l] = tab.level_tile_begin[l];
    sa.barrier = counters + many_sync_base(nseg);
    gridDim.x = (unsigned)nwg;
    ManyArgs a;
    memset(&a, 0, sizeof a);
    a.in = in;
    a.out = out;
    a.segs = segs.data();
    a.tile_seg = tab.tile_seg.data();
    a.counters = counters;
    a.total_items = items;
    a.nseg = nseg;
    a.dir = -1;
    // polls before a wait gives up (EMU_SPIN_LIMIT overrides, for the test of
    // an unmet dependency)
    a.spin_limit = getenv("EMU_SPIN_LIMIT") ? atoi(getenv("EMU_SPIN_LIMIT")) : 1 << 22;
    blockDim.x = threads;
    auto body = [&](V* lds) {
        if (sync) many_sync_body<V>(a, sa, lds, EmuLevelDispatch<V>{});
        else many_body<V>(a, lds, EmuDispatch<V>{});
    };
    if (levels) {
        // one workgroup per tile, the levels one after the other; with
        // EMU_GROUP_BYTES the grouped schedule of the library's own builder
        // (each group's levels before the next group's, through the tile map)
        std::vector<V> lds(lds_elems);
        bool okl = true;
        std::vector<int64_t> ranges;
        ManyGroups grp;
        if (const char* gb = getenv("EMU_GROUP_BYTES")) {
            build_many_groups(gd, tab, (int64_t)sizeof(V), atoll(gb), &grp);
            a.tile_map = grp.map.data();
            ranges = grp.ranges;
            std::printf("GROUPS %d\n", grp.groups);
        } else {
            ranges.assign(tab.level_tile_begin, tab.level_tile_begin + 4);
        }
        for (size_t r = 0; r + 1 < ranges.size(); ++r) {
            const int64_t begin = ranges[r];
            gridDim.x = (unsigned)(ranges[r + 1] - begin);
            for (unsigned b = 0; b < gridDim.x; ++b) {
                blockIdx.x = b;
                okl = run_block(threads, [&](int) {
                    if (all_cases) many_level_body<V>(a, begin, lds.data(), EmuLevelDispatchAll<V>{});
                    else many_level_body<V>(a, begin, lds.data(), EmuLevelDispatch<V>{});
                }) && okl;
            }
        }
        if (!okl) {
            std::printf("FAIL barrier\n");
            return 1;
        }
        std::printf("OK %lld tiles\n", (long long)tab.level_tile_begin[3]);
        for (int64_t i = 0; i < total; ++i) std::printf("%.17g %.17g\n", (double)out[i].x, (double)out[i].y);
        return 0;
    }
    std::vector<pid_t> kids;
    for (int wg = 1; wg < nwg; ++wg) {
        const pid_t pid = fork();
        if (pid == 0) {
            blockIdx.x = (unsigned)wg;
            std::vector<V> lds(lds_elems);
            const bool okc = run_block(threads, [&](int) { body(lds.data()); });
            _exit(okc ? 0 : 1);
        }
        kids.push_back(pid);
    }
    blockIdx.x = 0;
    std::vector<V> lds(lds_elems);
    bool ok = run_block(threads, [&](int) { body(lds.data()); });
    for (pid_t pid : kids) {
        int st = 0;
        waitpid(pid, &st, 0);
        if (!WIFEXITED(st) || WEXITSTATUS(st) != 0) ok = false;
    }
    if (!ok || counters[1]) {
        std::printf("FAIL barrier_ok=%d err=%u waiting_items=%lld\n", (int)ok, counters[1], (long long)waiting_items);
        return 1;
    }
    for (int l = 0; sync && l < 2; ++l)   // every workgroup arrived at both level barriers
        if (sa.barrier[l * kManySyncStride] != (unsigned)nwg) {
            std::printf("FAIL barrier %d arrivals %u of %d\n", l, sa.barrier[l * kManySyncStride], nwg);
            return 1;
        }
    for (int s = 0; !sync && s < nseg; ++s)   // a grid's last pass publishes nothing
        if (counters[kManyCounterBase + s] != (segs[s].last ? 0u : (unsigned)segs[s].nitems)) {
            std::printf("FAIL segment %d done %u of %d\n", s, counters[kManyCounterBase + s], segs[s].nitems);
            return 1;
        }
    std::printf("OK %lld items\n", (long long)items);
    for (int64_t i = 0; i < total; ++i) std::printf("%.17g %.17g\n", (double)out[i].x, (double)out[i].y);
    return 0;
}

template <typename V>
static int do_pass(int argc, char** argv) {
    if (argc < 10) return 2;
    const int kid = atoi(argv[3]);
    const int L = atoi(argv[4]);
    const int64_t M1 = atoll(argv[5]), M2 = atoll(argv[6]);
    const int logW = atoi(argv[7]), logP = atoi(argv[8]);
    const int tpl = atoi(argv[9]);
    // optional: transposing mode (2 or 3) and its row map X, Y
    const int tmode = argc > 10 ? atoi(argv[10]) : 0;
    const int64_t X = argc > 12 ? atoll(argv[11]) : 1, Y = argc > 12 ? atoll(argv[12]) : 1;
    if (tmode != 0 && (tmode < 2 || tmode > 3 || X * Y != M2)) return 2;
    const int64_t total = M1 * L * M2;
    std::vector<V> in(total), out(total);
    for (int64_t i = 0; i < total; ++i) {
        in[i].x = (decltype(in[i].x))std::sin(0.37 * (double)i + 0.1);
        in[i].y = (decltype(in[i].y))std::cos(0.91 * (double)i);
        out[i].x = out[i].y = 0;
    }
    std::vector<V> tw;
    twiddles(tw, L);
    PassArgs a;
    memset(&a, 0, sizeof a);
    a.in = in.data();
    a.out = out.data();
    a.tw = tw.data();
    a.nlines = M1 * M2;
    a.M2 = M2;
    a.lpm = M2;
    a.blk_logw = -1;
    // EMU_BLK="logw ld off": a strided pass restricted to the column block of
    // 2^logw columns starting at column off of every row of ld columns
    if (const char* blk = getenv("EMU_BLK")) {
        int lw = -1;
        long long ld = 0, off = 0;
        if (sscanf(blk, "%d %lld %lld", &lw, &ld, &off) != 3 || lw < 0 || ld < 1 || M2 % ld != 0 ||
            off + (1LL << lw) > ld || tmode != 0)
            return 2;
        a.blk_logw = lw;
        a.blk_ld = ld;
        a.blk_off = off;
        a.lpm = M2 / ld * (1LL << lw);
        a.nlines = M1 * a.lpm;
    }
    a.logW = logW;
    a.mode = tmode ? tmode : (M2 > 1 ? 1 : 0);
    a.X = X;
    a.Y = Y;
    a.scale = 1.0;
    const int W = 1 << logW;
    const int threads = W * tpl;
    // exactly the LDS the host launches the tile with: ASan flags any access beyond it
    const int P = M2 > 1 ? 1 << logP : 1;
    std::vector<V> lds((size_t)(tmode ? tile_lds_elems_transpose(W, L, P) : tile_lds_elems(W, L, P)));
    blockDim.x = threads;
    const int64_t nblocks = (a.nlines + W - 1) / W;
    for (int64_t blk = 0; blk < nblocks; ++blk) {
        blockIdx.x = (unsigned)blk;
        if (!run_block(threads, [&](int) { EmuDispatchPlain<V>{}(kid, P, a, lds.data(), blk << logW); })) {
            std::printf("FAIL barrier in tile %lld\n", (long long)blk);
            return 1;
        }
    }
    std::printf("OK %lld tiles\n", (long long)nblocks);
    for (int64_t i = 0; i < total; ++i) std::printf("%.17g %.17g\n", (double)out[i].x, (double)out[i].y);
    return 0;
}

// Runs a kernel body for every (block, thread) of a grid, one at a time (the
// exchange code has no barriers).
static void run_grid(unsigned blocks, unsigned threads, const std::function<void()>& body) {
    gridDim.x = blocks;
    blockDim.x = threads;
    for (unsigned b = 0; b < blocks; ++b) {
        blockIdx.x = b;
        for (unsigned t = 0; t < threads; ++t) {
            threadIdx.x = t;
            body();
        }
    }
}

// The pack kernel's body with its LDS tile (a static: shared by the
// emulated threads of one workgroup).
static void emu_pack(const PackArgs& a) {
    __shared__ PackShared<double2> sh;
    pack_tile<double2>(a, sh);
}

// Blocks one after the other, the threads of each concurrently with a
// barrier; false if a block's threads passed different numbers of barriers.
static bool run_grid_sync(unsigned blocks, unsigned threads, const std::function<void()>& body) {
    gridDim.x = blocks;
    blockDim.x = threads;
    bool ok = true;
    for (unsigned b = 0; b < blocks; ++b) {
        blockIdx.x = b;
        ok = run_block((int)threads, [&](int) { body(); }) && ok;
    }
    return ok;
}

// One exchange as dist.hip runs it: the library's tables (forward for the
// chunk sizes and places, reverse for the positions), pack per process with
// its own chunk into the receive array or straight into O_out, copies of the
// other chunks, unpack of every process's lines (all chunks at once or chunk
// by chunk).
static int do_route(int argc, char** argv) {
    if (argc < 9) return 2;
    const int64_t dims[3] = {atoll(argv[2]), atoll(argv[3]), atoll(argv[4])};
    const int np = atoi(argv[5]), in_order = atoi(argv[6]), out_order = atoi(argv[7]);
    const bool per_chunk = atoi(argv[8]) != 0;
    std::vector<int64_t> st[3];
    for (int o = 0; o < 3; ++o) {
        st[o].resize(np + 1);
        dist_line_starts(dims, o, np, st[o].data());
    }
    const int64_t* is = st[in_order].data();
    const int64_t* os = st[out_order].data();
    ExchangeTables t, rev;
    if (!build_exchange_tables(dims, np, in_order, out_order, is, os, &t) ||
        !build_exchange_tables(dims, np, out_order, in_order, os, is, &rev)) {
        std::printf("FAIL tables\n");
        return 1;
    }
    const int64_t N = dims[0] * dims[1] * dims[2];
    // exactly N elements per array: AddressSanitizer flags any access beyond
    std::vector<double2> in(N), send(N), recv(N), out(N);
    for (int64_t i = 0; i < N; ++i) {
        in[i].x = (double)i;
        in[i].y = 0.0;
        out[i].x = -1.0;
        out[i].y = 0.0;
    }
    ReverseTables rt;
    memset(&rt, 0, sizeof rt);
    rt.klo = rev.klo.data();
    rt.cnt = rev.cnt.data();
    rt.pre = rev.pre.data();
    rt.in_start = is;
    rt.nm = rev.in_n[1];
    rt.base_mul = rev.base_mul;
    rt.step = rev.step;
    rt.nq = rev.nq;
    rt.q_slowest = rev.q_slowest;
    const int u_axis = t.out_ax[2];
    if (u_axis != t.in_ax[0] && u_axis != t.in_ax[1]) {
        std::printf("FAIL axes\n");
        return 1;
    }
    bool ok = true;
    std::vector<char> direct(np);
    for (int sp = 0; sp < np; ++sp) {
        direct[sp] = t.count[(size_t)sp * np + sp] == (os[sp + 1] - os[sp]) * t.out_n[2];
        PackArgs a;
        memset(&a, 0, sizeof a);
        a.from = in.data();
        a.send = send.data();
        a.self = direct[sp] ? out.data() + os[sp] * t.out_n[2] : recv.data() + t.rdispl[(size_t)sp * np + sp];
        a.sdispl = t.sdispl.data();
        a.out_start = os;
        a.rev = rt;
        for (int i = 0; i < 3; ++i) {
            a.in_n[i] = t.in_n[i];
            a.out_n[i] = t.out_n[i];
            a.in_ax[i] = t.in_ax[i];
            a.out_ax[i] = t.out_ax[i];
        }
        a.u_slowest = u_axis == t.in_ax[0] ? 1 : 0;
        a.np = np;
        a.src = sp;
        a.line_begin = is[sp];
        a.line_end = is[sp + 1];
        const int64_t nm = a.in_n[1];
        const int64_t lo = a.line_begin / nm, hi = (a.line_end - 1) / nm + 1;
        if (a.u_slowest) { a.u_lo = lo; a.u_n = hi - lo; a.v_lo = 0; a.v_n = nm; }
        else { a.v_lo = lo; a.v_n = hi - lo; a.u_lo = 0; a.u_n = nm; }
        a.u_tiles = (a.u_n + kPackTile - 1) / kPackTile;
        a.k_tiles = (a.in_n[2] + kPackTile - 1) / kPackTile;
        ok = run_grid_sync((unsigned)(a.v_n * a.u_tiles * a.k_tiles), kPackThreads, [&] { emu_pack(a); }) && ok;
    }
    for (int sp = 0; sp < np; ++sp)
        for (int d = 0; d < np; ++d) {
            if (sp == d) continue;   // the own chunk is already in place
            CopyDesc c;
            c.from = t.sdispl[(size_t)sp * np + d];
            c.to = t.rdispl[(size_t)d * np + sp];
            c.n = t.count[(size_t)sp * np + d];
            if (c.n) run_grid(2, kCopyThreads, [&] { copy_chunk(send.data(), recv.data(), c); });
        }
    for (int d = 0; d < np; ++d) {
        if (direct[d]) continue;
        for (int sp = per_chunk ? 0 : -1; sp < (per_chunk ? np : 0); ++sp) {
            GatherArgs a;
            memset(&a, 0, sizeof a);
            a.recv = recv.data();
            a.to = out.data();
            a.rdispl = t.rdispl.data();
            a.rev = rt;
            a.nf = t.out_n[2];
            a.line_begin = os[d];
            a.line_end = os[d + 1];
            a.np = np;
            a.dst = d;
            a.src_only = sp;
            // fewer waves than lines: the line loop is exercised
            run_grid(2, kGatherThreads, [&] { gather_lines<double2>(a); });
        }
    }
    if (!ok) {
        std::printf("FAIL barrier\n");
        return 1;
    }
    std::printf("OK\n");
    for (int sp = 0; sp < np; ++sp) {
        for (int d = 0; d < np; ++d) std::printf("%lld ", (long long)t.count[(size_t)sp * np + d]);
        std::printf("\n");
    }
    for (int64_t i = 0; i < N; ++i) std::printf("%lld\n", (long long)out[i].x);
    return 0;
}

int main(int argc, char** argv) {
    if (argc < 3) return 2;
    const std::string mode = argv[1];
    if (mode == "route") return do_route(argc, argv);
    const int dtype = atoi(argv[2]);
    if (mode == "many") return dtype == 0 ? do_many<double2>(argc, argv, false) : do_many<float2>(argc, argv, false);
    if (mode == "sync") return dtype == 0 ? do_many<double2>(argc, argv, true) : do_many<float2>(argc, argv, true);
    if (mode == "tables")
        return dtype == 0 ? do_many<double2>(argc, argv, false, false, true)
                          : do_many<float2>(argc, argv, false, false, true);
    if (mode == "levels")
        return dtype == 0 ? do_many<double2>(argc, argv, false, true) : do_many<float2>(argc, argv, false, true);
    if (mode == "levels_all")
        return dtype == 0 ? do_many<double2>(argc, argv, false, true, false, true)
                          : do_many<float2>(argc, argv, false, true, false, true);
    if (mode == "pass") return dtype == 0 ? do_pass<double2>(argc, argv) : do_pass<float2>(argc, argv);
    return 2;
}
