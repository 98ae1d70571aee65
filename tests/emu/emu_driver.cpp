// emu_driver.cpp -- runs the library's tile code (pass_tile) and the
// persistent batch loop (many_body) for one workgroup on CPU threads.
//
//   emu_driver pass <dtype 0|1> <kid> <L> <M1> <M2> <logW> <logP> <TPL>
//       one stand-alone axis pass (kernel case kid of the executor's table,
//       plain stores) over a [M1][L][M2] view of synthetic data, tile by tile
//       with W*TPL threads each (strided lines with LDS exchanges in 2^logP
//       parts when M2 > 1); prints the forward-transformed data as text
//   emu_driver many <dtype> <nwg> <threads> <nseg> <segments...> <total>
//       the persistent loop over a segment table, run by nwg workgroups at
//       once: each workgroup is a forked process of `threads` CPU threads;
//       buffers and counters live in shared memory
//   emu_driver sync <dtype> <nwg> <threads> <nseg> <segments + level...> <total>
//       the level-synchronous persistent body (grid barriers between levels)
//       over the batch executor's cases, nwg workgroups at once
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
static int do_many(int argc, char** argv, bool sync) {
    // many|sync <dtype> <nwg> <threads> <nseg> then per segment:
    //   L kid logW mode nlines M2 ntiles first last dep elem_off tiles_per_item [level (sync)]
    // then <total_elems>
    int k = 3;
    const int nwg = atoi(argv[k++]);
    const int threads = atoi(argv[k++]);
    const int nseg = atoi(argv[k++]);
    std::vector<ManySeg> segs(nseg);
    std::vector<int> seg_level(nseg, 0);
    std::vector<std::vector<V>> tws(nseg);
    int64_t items = 0;
    size_t lds_elems = 0;
    for (int s = 0; s < nseg; ++s) {
        ManySeg& g = segs[s];
        memset(&g, 0, sizeof g);
        const int L = atoi(argv[k++]);
        g.kid = atoi(argv[k++]);
        g.logW = atoi(argv[k++]);
        g.mode = atoi(argv[k++]);
        g.nlines = atoll(argv[k++]);
        g.M2 = atoll(argv[k++]);
        g.ntiles = atoi(argv[k++]);
        g.first = atoi(argv[k++]);
        g.last = atoi(argv[k++]);
        g.dep = atoi(argv[k++]);
        g.elem_off = atoll(argv[k++]);
        g.tiles_per_item = atoi(argv[k++]);
        if (sync) seg_level[s] = atoi(argv[k++]);
        g.nitems = (g.ntiles + g.tiles_per_item - 1) / g.tiles_per_item;
        g.scale_bwd = 1.0;
        g.item_base = items;
        items += g.nitems;
        twiddles(tws[s], L);
        g.tw = tws[s].data();
        lds_elems = std::max(lds_elems, (size_t)tile_lds_elems(1 << g.logW, L));
    }
    const int64_t total = atoll(argv[k++]);
    // (level, case) groups of the level-synchronous form, built as the library does
    // as many cases as the executor has (the kernel walks all of them)
    int ncases = sync ? EmuSync<V>::ncases : 0;
    for (const ManySeg& g : segs) ncases = std::max(ncases, g.kid + 1);
    std::vector<ManyGroup> groups((size_t)3 * ncases);
    std::vector<int> gseg;
    for (int lvl = 0; lvl < 3; ++lvl) {
        int64_t rot = 0;
        for (int c = 0; c < ncases; ++c) {
            ManyGroup& gr = groups[(size_t)lvl * ncases + c];
            gr.seg_begin = (int)gseg.size();
            gr.ntiles = 0;
            gr.rot = rot;
            for (int i = 0; i < nseg; ++i) {
                if (seg_level[i] != lvl || segs[i].kid != c) continue;
                segs[i].group_tile_base = gr.ntiles;
                gr.ntiles += segs[i].ntiles;
                gseg.push_back(i);
            }
            gr.seg_end = (int)gseg.size();
            rot += gr.ntiles;
        }
    }
    // shared between the workgroup processes: buffers, counters, two level barriers
    const size_t bytes = sizeof(V) * 2 * (size_t)total + sizeof(unsigned) * (kManyCounterBase + nseg + 2);
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
    for (int i = 0; i < kManyCounterBase + nseg + 2; ++i) counters[i] = 0u;
    ManySyncArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.groups = groups.data();
    sa.gseg = gseg.data();
    sa.barrier = counters + kManyCounterBase + nseg;
    sa.ncases = ncases;
    gridDim.x = (unsigned)nwg;
    ManyArgs a;
    memset(&a, 0, sizeof a);
    a.in = in;
    a.out = out;
    a.segs = segs.data();
    a.counters = counters;
    a.total_items = items;
    a.nseg = nseg;
    a.dir = -1;
    // polls before a wait gives up (EMU_SPIN_LIMIT overrides, for the test of
    // an unmet dependency)
    a.spin_limit = getenv("EMU_SPIN_LIMIT") ? atoi(getenv("EMU_SPIN_LIMIT")) : 1 << 22;
    blockDim.x = threads;
    auto body = [&](V* lds) {
        if (sync) EmuSync<V>::body(a, sa, lds);
        else many_body<V>(a, lds, EmuDispatch<V>{});
    };
    std::vector<pid_t> kids;
    for (int wg = 1; wg < nwg; ++wg) {
        const pid_t pid = fork();
        if (pid == 0) {
            blockIdx.x = (unsigned)wg;
            std::vector<V> lds(lds_elems + 64);
            const bool okc = run_block(threads, [&](int) { body(lds.data()); });
            _exit(okc ? 0 : 1);
        }
        kids.push_back(pid);
    }
    blockIdx.x = 0;
    std::vector<V> lds(lds_elems + 64);
    bool ok = run_block(threads, [&](int) { body(lds.data()); });
    for (pid_t pid : kids) {
        int st = 0;
        waitpid(pid, &st, 0);
        if (!WIFEXITED(st) || WEXITSTATUS(st) != 0) ok = false;
    }
    if (!ok || counters[1]) {
        std::printf("FAIL barrier_ok=%d err=%u\n", (int)ok, counters[1]);
        return 1;
    }
    for (int l = 0; sync && l < 2; ++l)   // every workgroup arrived at both level barriers
        if (counters[kManyCounterBase + nseg + l] != (unsigned)nwg) {
            std::printf("FAIL barrier %d arrivals %u of %d\n", l, counters[kManyCounterBase + nseg + l], nwg);
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
    ExchangeTables t;
    if (!build_exchange_tables(dims, np, in_order, out_order, st[in_order].data(), st[out_order].data(), &t)) {
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
    RouteArgs r;
    memset(&r, 0, sizeof r);
    for (int i = 0; i < 3; ++i) {
        r.in_n[i] = t.in_n[i];
        r.out_n[i] = t.out_n[i];
        r.in_ax[i] = t.in_ax[i];
        r.out_ax[i] = t.out_ax[i];
    }
    r.sdispl = t.sdispl.data();
    r.rdispl = t.rdispl.data();
    r.klo = t.klo.data();
    r.cnt = t.cnt.data();
    r.pre = t.pre.data();
    r.out_start = st[out_order].data();
    r.base_mul = t.base_mul;
    r.step = t.step;
    r.nq = t.nq;
    r.q_slowest = t.q_slowest;
    r.np = np;
    const unsigned blocks = 3;   // fewer blocks than lines: the grid-stride loop is exercised
    for (int sp = 0; sp < np; ++sp) {
        RouteArgs a = r;
        a.from = in.data();
        a.to = send.data();
        a.src = sp;
        a.dst_only = -1;
        a.unpack = 0;
        a.line_begin = st[in_order][sp];
        a.line_end = st[in_order][sp + 1];
        run_grid(blocks, kRouteThreads, [&] { route_lines<double2>(a); });
    }
    for (int sp = 0; sp < np; ++sp)
        for (int d = 0; d < np; ++d) {
            CopyDesc c;
            c.from = t.sdispl[(size_t)sp * np + d];
            c.to = t.rdispl[(size_t)d * np + sp];
            c.n = t.count[(size_t)sp * np + d];
            if (c.n) run_grid(2, kCopyThreads, [&] { copy_chunk(send.data(), recv.data(), c); });
        }
    for (int sp = 0; sp < np; ++sp)
        for (int d = per_chunk ? 0 : -1; d < (per_chunk ? np : 0); ++d) {
            RouteArgs a = r;
            a.from = recv.data();
            a.to = out.data();
            a.src = sp;
            a.dst_only = d;
            a.unpack = 1;
            a.line_begin = st[in_order][sp];
            a.line_end = st[in_order][sp + 1];
            run_grid(blocks, kRouteThreads, [&] { route_lines<double2>(a); });
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
    if (mode == "pass") return dtype == 0 ? do_pass<double2>(argc, argv) : do_pass<float2>(argc, argv);
    return 2;
}
