// dist.hip -- the paper's distributed calculation flow (Duy & Ozaki, Sec. 2
// and Sec. 3.1.1) run by Np virtual processes on one GPU.
//
// Process p owns the Eq. 2 block of the linear index of the order the data is
// held in: [f(p), f(p+1)) with f over that order's leading dimensions (whole
// N2 x N3 planes when Np <= N1, whole N3-lines when N1 < Np <= N1 N2).  Every
// block is a contiguous range of that order's linear index, so the processes'
// local arrays are consecutive slices of one global array in that order.  The
// forward flow is
//   1. the 1-D transform of every local line along c (abc order, c fastest),
//   2. the transpose abc -> cab: pack, communicate, unpack,
//   3. the 1-D transform along b (cab order),
//   4. the transpose cab -> cba,
//   5. the 1-D transform along a (cba order),
// and the data finishes in the cba decomposition.  The backward flow runs
// the same steps in reverse with the conjugate roots of unity.
//
// One exchange (O_in -> O_out): each element of process src moves to the
// process dst that owns its linear index in O_out.
//   pack         src's elements grouped by dst into consecutive chunks of
//                src's send slice, each chunk in dst's O_out order (a tiled
//                transpose through LDS); src's own chunk goes straight to
//                its place in the receive array -- or into the O_out array
//                itself when src receives nothing from anyone else;
//   communicate  chunk (src, dst), src != dst, copied from src's send slice
//                into dst's receive slice, chunks ordered by src -- the six
//                methods of Sec. 3.2.1 are six ways of issuing and waiting
//                for these copies;
//   unpack       dst's O_out lines filled from the received chunks: every
//                line is a sequence of runs, one per sending process, each a
//                contiguous piece of that process's chunk.
// Positions need no index table: along an O_out line (its fastest axis, k')
// the O_in line index is base + k'*step, increasing, so the elements of one
// O_out line that come from one process form one run; base depends on one
// coordinate q of the line, so the number of elements a process contributes
// to the lines before line m is a closed form over per-q counts and their
// prefix sums (the tables of the reverse exchange O_out -> O_in).  The
// chunk sizes (the elements each process sends each other one) come from
// the same construction in the forward direction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/offt.h"
#include "offt_internal.h"
#include "plan_impl.h"
#include "dist_device.hpp"
#include "dist_tables.hpp"

namespace offt {

constexpr int kDistMaxProcs = 64;
constexpr int kDistMethods = 6;
constexpr int kGatherMaxBlocks = 16384;

// The kernels of one exchange (device code in dist_device.hpp).
template <typename V>
__global__ void __launch_bounds__(kPackThreads) pack_kernel(PackArgs a) {
    __shared__ PackShared<V> sh;
    pack_tile<V>(a, sh);
}

template <typename V>
__global__ void __launch_bounds__(kGatherThreads) gather_kernel(GatherArgs a) {
    gather_lines<V>(a);
}

template <typename V>
__global__ void __launch_bounds__(kCopyThreads) copy_chunks_kernel(const V* __restrict__ send, V* __restrict__ recv,
                                                                   const CopyDesc* __restrict__ desc) {
    copy_chunk(send, recv, desc[blockIdx.y]);
}

// A line of one point: its transform is the identity, with the backward
// transform's conjugations and scaling still applied.
template <typename V>
__global__ void __launch_bounds__(kCopyThreads) unit_lines_kernel(const V* in, V* out,
                                                                  int64_t n, int conj_in, int conj_out, double scale) {
    using S = decltype(V{}.x);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        V x = in[i];
        if (conj_in != conj_out) x.y = -x.y;
        x.x *= (S)scale;
        x.y *= (S)scale;
        out[i] = x;
    }
}

// One exchange O_in -> O_out of the plan's processes.
struct Exchange {
    int in_order = 0, out_order = 0;
    std::vector<int64_t> count;        // [src * np + dst]
    std::vector<int64_t> sdispl, rdispl;
    std::vector<char> direct;          // [proc]: proc receives only from itself (its pack writes O_out)
    PackArgs pack{};                   // device table pointers and shape fields
    GatherArgs gather{};
    int64_t max_chunk = 0;
    // device descriptors of the chunk copies, per launch of each method
    CopyDesc* d_desc = nullptr;
    struct Launch {
        int first, n;                  // descriptors [first, first + n)
        int src, dst;                  // the chunk's processes (one-chunk launches), else -1
    };
    std::vector<Launch> launches[kDistMethods];
    std::vector<int> group_end[kDistMethods];   // block methods: launches that end each group
};

struct DistState {
    int np = 1;
    int method = OFFT_COMM_ISEND_WAITSOME;
    int block = 32;
    float method_ms[kDistMethods] = {-1, -1, -1, -1, -1, -1};
    int64_t line_start[3][kDistMaxProcs + 1] = {};   // first line of each process per order
    Exchange fwd[2], bwd[2];
    PassPlan pass[3][kDistMaxProcs];                 // per order, per process: the line transforms
    void* work = nullptr;
    void* send = nullptr;
    void* recv = nullptr;
    hipStream_t comm = nullptr;
    hipEvent_t ev_start = nullptr, ev_group = nullptr;
    std::vector<hipEvent_t> ev_chunk;                // one per chunk (src * np + dst)
};

static int dist_alloc(offt_plan_s* p, size_t bytes, void** out) {
    if (hipMalloc(out, bytes ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return OFFT_ERR_OUT_OF_MEMORY;
    }
    p->allocs.push_back(*out);
    p->alloc_bytes.push_back(bytes);
    return OFFT_SUCCESS;
}

template <typename T>
static int upload(offt_plan_s* p, const std::vector<T>& v, const T** out, hipStream_t s) {
    void* d = nullptr;
    const int rc = dist_alloc(p, sizeof(T) * std::max<size_t>(v.size(), 1), &d);
    if (rc) return rc;
    if (!v.empty() && hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return OFFT_ERR_HIP;
    *out = static_cast<const T*>(d);
    return OFFT_SUCCESS;
}

// Builds one exchange: run tables, chunk counts and displacements
// (dist_tables.hpp), and the copy launches of every method.
static int build_exchange(offt_plan_s* p, DistState* ds, int in_order, int out_order, Exchange* ex, hipStream_t s) {
    const int np = ds->np;
    ex->in_order = in_order;
    ex->out_order = out_order;
    const int64_t* in_start = ds->line_start[in_order];
    const int64_t* out_start = ds->line_start[out_order];
    ExchangeTables t, rev;
    if (!build_exchange_tables(p->dims, np, in_order, out_order, in_start, out_start, &t) ||
        !build_exchange_tables(p->dims, np, out_order, in_order, out_start, in_start, &rev))
        return OFFT_ERR_BAD_PLAN;
    // the pack's tiles run along the O_in axis that is O_out's fastest
    const int u_axis = t.out_ax[2];
    if (u_axis != t.in_ax[0] && u_axis != t.in_ax[1]) return OFFT_ERR_BAD_PLAN;
    ex->count = t.count;
    ex->sdispl = t.sdispl;
    ex->rdispl = t.rdispl;
    ex->max_chunk = t.max_chunk;
    ex->direct.assign(np, 0);
    for (int d = 0; d < np; ++d)
        ex->direct[d] = t.count[(size_t)d * np + d] == (out_start[d + 1] - out_start[d]) * t.out_n[2];
    ReverseTables rt;
    memset(&rt, 0, sizeof rt);
    rt.nm = rev.in_n[1];
    rt.base_mul = rev.base_mul;
    rt.step = rev.step;
    rt.nq = rev.nq;
    rt.q_slowest = rev.q_slowest;
    std::vector<int64_t> is(in_start, in_start + np + 1), os(out_start, out_start + np + 1);
    int rc = upload(p, rev.klo, &rt.klo, s);
    if (!rc) rc = upload(p, rev.cnt, &rt.cnt, s);
    if (!rc) rc = upload(p, rev.pre, &rt.pre, s);
    if (!rc) rc = upload(p, is, &rt.in_start, s);
    PackArgs& pa = ex->pack;
    memset(&pa, 0, sizeof pa);
    pa.rev = rt;
    for (int i = 0; i < 3; ++i) {
        pa.in_n[i] = t.in_n[i];
        pa.out_n[i] = t.out_n[i];
        pa.in_ax[i] = t.in_ax[i];
        pa.out_ax[i] = t.out_ax[i];
    }
    pa.u_slowest = u_axis == t.in_ax[0] ? 1 : 0;
    pa.np = np;
    GatherArgs& ga = ex->gather;
    memset(&ga, 0, sizeof ga);
    ga.rev = rt;
    ga.nf = t.out_n[2];
    ga.np = np;
    if (!rc) rc = upload(p, t.sdispl, &pa.sdispl, s);
    if (!rc) rc = upload(p, os, &pa.out_start, s);
    if (!rc) rc = upload(p, t.rdispl, &ga.rdispl, s);
    if (rc) return rc;
    // copy descriptors, laid out per method so that each launch covers
    // consecutive descriptors; empty chunks and a process's own chunk are
    // not sent
    std::vector<CopyDesc> desc;
    auto sent = [&](int sp, int d) { return sp != d && ex->count[(size_t)sp * np + d] != 0; };
    auto chunk = [&](int sp, int d) {
        CopyDesc c;
        c.from = ex->sdispl[(size_t)sp * np + d];
        c.to = ex->rdispl[(size_t)d * np + sp];
        c.n = ex->count[(size_t)sp * np + d];
        return c;
    };
    const int B = std::max(1, std::min(ds->block, np));
    const int ngroups = (np + B - 1) / B;
    for (int m = 0; m < kDistMethods; ++m) {
        auto one = [&](int sp, int d) {
            if (!sent(sp, d)) return;
            ex->launches[m].push_back({(int)desc.size(), 1, sp, d});
            desc.push_back(chunk(sp, d));
        };
        if (m == OFFT_COMM_ISEND_WAITALL || m == OFFT_COMM_ISEND_WAITSOME) {
            // every process posts a send to every other process at once
            for (int sp = 0; sp < np; ++sp)
                for (int d = 0; d < np; ++d) one(sp, d);
        } else if (m == OFFT_COMM_ALLTOALLV) {
            // one collective call over every chunk
            const int first = (int)desc.size();
            for (int sp = 0; sp < np; ++sp)
                for (int d = 0; d < np; ++d)
                    if (sent(sp, d)) desc.push_back(chunk(sp, d));
            if ((int)desc.size() > first) ex->launches[m].push_back({first, (int)desc.size() - first, -1, -1});
        } else if (m == OFFT_COMM_ISEND_WAITALL_BLOCK || m == OFFT_COMM_ISEND_WAITSOME_BLOCK) {
            // group g: every process exchanges with the processes of group g
            for (int g = 0; g < ngroups; ++g) {
                for (int sp = 0; sp < np; ++sp)
                    for (int d = g * B; d < std::min(np, (g + 1) * B); ++d) one(sp, d);
                ex->group_end[m].push_back((int)ex->launches[m].size());
            }
        } else {
            // step i >= 1: process myid sends to myid + i and receives from
            // myid - i (step 0, the own chunk, needs no copy)
            for (int i = 1; i < np; ++i) {
                const int first = (int)desc.size();
                for (int sp = 0; sp < np; ++sp) {
                    const int d = (sp + i) % np;
                    if (sent(sp, d)) desc.push_back(chunk(sp, d));
                }
                if ((int)desc.size() > first) ex->launches[m].push_back({first, (int)desc.size() - first, -1, i});
            }
        }
    }
    if (desc.empty()) return OFFT_SUCCESS;   // every process keeps its data
    const CopyDesc* dd = nullptr;
    rc = upload(p, desc, &dd, s);
    ex->d_desc = const_cast<CopyDesc*>(dd);
    return rc;
}

void release_dist(offt_plan_s* p) {
    DistState* ds = p->dist;
    if (!ds) return;
    for (hipEvent_t e : ds->ev_chunk)
        if (e) (void)hipEventDestroy(e);
    if (ds->ev_start) (void)hipEventDestroy(ds->ev_start);
    if (ds->ev_group) (void)hipEventDestroy(ds->ev_group);
    if (ds->comm) (void)hipStreamDestroy(ds->comm);
    delete ds;
    p->dist = nullptr;
}

// Pack of process sp: its O_in lines of `from` into the send array (chunks to
// the others) and its own chunk into `self`.
static hipError_t launch_pack(const offt_plan_s* p, const Exchange& ex, int sp, const void* from, void* self,
                              hipStream_t s) {
    const DistState* ds = p->dist;
    PackArgs a = ex.pack;
    a.from = from;
    a.send = ds->send;
    a.self = self;
    a.src = sp;
    a.line_begin = ds->line_start[ex.in_order][sp];
    a.line_end = ds->line_start[ex.in_order][sp + 1];
    if (a.line_end <= a.line_begin) return hipSuccess;
    const int64_t nm = a.in_n[1];
    const int64_t lo = a.line_begin / nm, hi = (a.line_end - 1) / nm + 1;   // slowest coordinates of the lines
    if (a.u_slowest) {
        a.u_lo = lo; a.u_n = hi - lo;
        a.v_lo = 0;  a.v_n = nm;
    } else {
        a.v_lo = lo; a.v_n = hi - lo;
        a.u_lo = 0;  a.u_n = nm;
    }
    a.u_tiles = (a.u_n + kPackTile - 1) / kPackTile;
    a.k_tiles = (a.in_n[2] + kPackTile - 1) / kPackTile;
    const int64_t blocks = a.v_n * a.u_tiles * a.k_tiles;
    if (blocks >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    if (p->dtype == OFFT_C2C_F64)
        hipLaunchKernelGGL(pack_kernel<double2>, dim3((unsigned)blocks), dim3(kPackThreads), 0, s, a);
    else
        hipLaunchKernelGGL(pack_kernel<float2>, dim3((unsigned)blocks), dim3(kPackThreads), 0, s, a);
    return hipGetLastError();
}

// Unpack of process d's O_out lines from the receive array into `to`; src
// >= 0: the chunk from that process only.
static hipError_t launch_unpack(const offt_plan_s* p, const Exchange& ex, int d, int src, void* to, hipStream_t s) {
    const DistState* ds = p->dist;
    GatherArgs a = ex.gather;
    a.recv = ds->recv;
    a.to = to;
    a.dst = d;
    a.src_only = src;
    a.line_begin = ds->line_start[ex.out_order][d];
    a.line_end = ds->line_start[ex.out_order][d + 1];
    const int64_t lines = a.line_end - a.line_begin;
    if (lines <= 0) return hipSuccess;
    constexpr int kWaves = kGatherThreads / 64;
    const unsigned blocks = (unsigned)std::min<int64_t>((lines + kWaves - 1) / kWaves, kGatherMaxBlocks);
    if (p->dtype == OFFT_C2C_F64)
        hipLaunchKernelGGL(gather_kernel<double2>, dim3(blocks), dim3(kGatherThreads), 0, s, a);
    else
        hipLaunchKernelGGL(gather_kernel<float2>, dim3(blocks), dim3(kGatherThreads), 0, s, a);
    return hipGetLastError();
}

static hipError_t launch_copies(const offt_plan_s* p, const Exchange& ex, const Exchange::Launch& L, hipStream_t s) {
    const DistState* ds = p->dist;
    const int64_t per = ex.max_chunk;
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((per + kCopyThreads * 4 - 1) / (kCopyThreads * 4),
                                                                       2048));
    const dim3 grid(gx, (unsigned)L.n);
    if (p->dtype == OFFT_C2C_F64)
        hipLaunchKernelGGL(copy_chunks_kernel<double2>, grid, dim3(kCopyThreads), 0, s,
                           static_cast<const double2*>(ds->send), static_cast<double2*>(ds->recv), ex.d_desc + L.first);
    else
        hipLaunchKernelGGL(copy_chunks_kernel<float2>, grid, dim3(kCopyThreads), 0, s,
                           static_cast<const float2*>(ds->send), static_cast<float2*>(ds->recv), ex.d_desc + L.first);
    return hipGetLastError();
}

// One exchange with the plan's method: pack every process's chunks, run the
// method's copies and waits, unpack into `to` (the global O_out array;
// `from` and `to` are different arrays).
static int run_exchange(const offt_plan_s* p, const Exchange& ex, int method, const void* from, void* to,
                        hipStream_t s) {
    DistState* ds = p->dist;
    const int np = ds->np;
    const size_t es = elem_size(p->dtype);
    for (int sp = 0; sp < np; ++sp) {
        // the own chunk: into the receive array, or straight into O_out
        void* self = ex.direct[sp] ? static_cast<char*>(to) + ds->line_start[ex.out_order][sp] * ex.gather.nf * es
                                   : static_cast<char*>(ds->recv) + ex.rdispl[(size_t)sp * np + sp] * es;
        if (launch_pack(p, ex, sp, from, self, s) != hipSuccess) return OFFT_ERR_HIP;
    }
    const auto& L = ex.launches[method];
    auto unpack_all = [&]() -> int {
        for (int d = 0; d < np; ++d)
            if (!ex.direct[d] && launch_unpack(p, ex, d, -1, to, s) != hipSuccess) return OFFT_ERR_HIP;
        return OFFT_SUCCESS;
    };
    // own chunks that are not already in place
    auto unpack_own = [&]() -> int {
        for (int d = 0; d < np; ++d)
            if (!ex.direct[d] && ex.count[(size_t)d * np + d] && launch_unpack(p, ex, d, d, to, s) != hipSuccess)
                return OFFT_ERR_HIP;
        return OFFT_SUCCESS;
    };
    // the communication stream starts after the packs
    auto fork = [&]() -> int {
        if (hipEventRecord(ds->ev_start, s) != hipSuccess || hipStreamWaitEvent(ds->comm, ds->ev_start, 0) != hipSuccess)
            return OFFT_ERR_HIP;
        return OFFT_SUCCESS;
    };
    if (method == OFFT_COMM_ALLTOALLV) {
        // one collective over every chunk, then the unpack
        for (const auto& l : L)
            if (launch_copies(p, ex, l, s) != hipSuccess) return OFFT_ERR_HIP;
        return unpack_all();
    }
    if (method == OFFT_COMM_SENDRECV) {
        // Np - 1 steps after the own chunk, each a blocking exchange with one
        // partner; the received chunk is unpacked before the next step
        int rc = unpack_own();
        for (const auto& l : L) {
            if (rc) return rc;
            if (launch_copies(p, ex, l, s) != hipSuccess) return OFFT_ERR_HIP;
            for (int sp = 0; sp < np; ++sp) {
                const int d = (sp + l.dst) % np;
                if (sp != d && ex.count[(size_t)sp * np + d] && launch_unpack(p, ex, d, sp, to, s) != hipSuccess)
                    return OFFT_ERR_HIP;
            }
        }
        return rc;
    }
    const bool some = method == OFFT_COMM_ISEND_WAITSOME || method == OFFT_COMM_ISEND_WAITSOME_BLOCK;
    const bool block = method == OFFT_COMM_ISEND_WAITALL_BLOCK || method == OFFT_COMM_ISEND_WAITSOME_BLOCK;
    std::vector<int> ends = block ? ex.group_end[method] : std::vector<int>{(int)L.size()};
    int rc = fork();
    // Waitsome: the own chunks are complete once packed
    if (rc == OFFT_SUCCESS && some) rc = unpack_own();
    int first = 0;
    for (int g = 0; g < (int)ends.size() && rc == OFFT_SUCCESS; ++g) {
        // the group's sends and receives are posted at once on the
        // communication stream; each chunk's arrival is an event
        for (int i = first; i < ends[g] && rc == OFFT_SUCCESS; ++i) {
            if (launch_copies(p, ex, L[i], ds->comm) != hipSuccess) rc = OFFT_ERR_HIP;
            else if (some && hipEventRecord(ds->ev_chunk[(size_t)L[i].src * np + L[i].dst], ds->comm) != hipSuccess)
                rc = OFFT_ERR_HIP;
        }
        if (rc != OFFT_SUCCESS) break;
        if (some) {
            // Waitsome: each chunk is unpacked as soon as it has arrived
            for (int i = first; i < ends[g] && rc == OFFT_SUCCESS; ++i) {
                const auto& l = L[i];
                if (hipStreamWaitEvent(s, ds->ev_chunk[(size_t)l.src * np + l.dst], 0) != hipSuccess ||
                    launch_unpack(p, ex, l.dst, l.src, to, s) != hipSuccess)
                    rc = OFFT_ERR_HIP;
            }
            // the next group is posted once this one is complete
            if (rc == OFFT_SUCCESS && block && g + 1 < (int)ends.size() &&
                (hipEventRecord(ds->ev_group, s) != hipSuccess || hipStreamWaitEvent(ds->comm, ds->ev_group, 0) != hipSuccess))
                rc = OFFT_ERR_HIP;
        } else {
            // Waitall: wait for every chunk of the group
            if (hipEventRecord(ds->ev_group, ds->comm) != hipSuccess ||
                (block && hipStreamWaitEvent(ds->comm, ds->ev_group, 0) != hipSuccess))
                rc = OFFT_ERR_HIP;
        }
        first = ends[g];
    }
    if (rc != OFFT_SUCCESS) return rc;
    if (!some) {
        if (hipStreamWaitEvent(s, ds->ev_group, 0) != hipSuccess) return OFFT_ERR_HIP;
        return unpack_all();
    }
    return OFFT_SUCCESS;
}

// The per-process line transforms of one order (step 1, 3 or 5).
static int run_lines(const offt_plan_s* p, int order, const void* in, void* out, int conj_in, int conj_out,
                     double scale, hipStream_t s) {
    const DistState* ds = p->dist;
    int64_t n[3];
    order_lengths(p->dims, order, n);
    const size_t es = elem_size(p->dtype);
    for (int sp = 0; sp < ds->np; ++sp) {
        const int64_t off = ds->line_start[order][sp] * n[2];
        const char* src = static_cast<const char*>(in) + off * es;
        char* dst = static_cast<char*>(out) + off * es;
        const PassPlan& pp = ds->pass[order][sp];
        if (n[2] == 1) {
            const int64_t cnt = pp.M1;
            if (conj_in == conj_out && scale == 1.0 && src == dst) continue;
            const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cnt + kCopyThreads - 1) / kCopyThreads, 4096));
            if (p->dtype == OFFT_C2C_F64)
                hipLaunchKernelGGL(unit_lines_kernel<double2>, dim3(blocks), dim3(kCopyThreads), 0, s,
                                   reinterpret_cast<const double2*>(src), reinterpret_cast<double2*>(dst), cnt, conj_in,
                                   conj_out, scale);
            else
                hipLaunchKernelGGL(unit_lines_kernel<float2>, dim3(blocks), dim3(kCopyThreads), 0, s,
                                   reinterpret_cast<const float2*>(src), reinterpret_cast<float2*>(dst), cnt, conj_in,
                                   conj_out, scale);
            if (hipGetLastError() != hipSuccess) return OFFT_ERR_HIP;
            continue;
        }
        if (launch_pass(pp, src, dst, conj_in, conj_out, scale, s) != hipSuccess) return OFFT_ERR_HIP;
    }
    return OFFT_SUCCESS;
}

// Conjugates n elements in place (the backward flow runs as conj(F(conj x));
// its intermediate states are reported unconjugated).
static int conj_in_place(const offt_plan_s* p, void* buf, int64_t n, hipStream_t s) {
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kCopyThreads - 1) / kCopyThreads, 4096));
    if (p->dtype == OFFT_C2C_F64)
        hipLaunchKernelGGL(unit_lines_kernel<double2>, dim3(blocks), dim3(kCopyThreads), 0, s,
                           static_cast<const double2*>(buf), static_cast<double2*>(buf), n, 1, 0, 1.0);
    else
        hipLaunchKernelGGL(unit_lines_kernel<float2>, dim3(blocks), dim3(kCopyThreads), 0, s,
                           static_cast<const float2*>(buf), static_cast<float2*>(buf), n, 1, 0, 1.0);
    return hipGetLastError() == hipSuccess ? OFFT_SUCCESS : OFFT_ERR_HIP;
}

// The first `steps` steps of the forward (dir < 0) or backward flow, `in` to
// `out`; after step k the global array of that step's order is in `out`
// (the unfinished later steps are not run).
int exec_dist(const offt_plan_s* p, int dir, int steps, const void* in, void* out, int method, int normalize,
              hipStream_t s) {
    const DistState* ds = p->dist;
    if (method < 0) method = ds->method;
    const bool bwd = dir > 0;
    const int64_t N = p->dims[0] * p->dims[1] * p->dims[2];
    const int norm = normalize < 0 ? p->normalize : normalize;
    const double scale = (bwd && norm) ? 1.0 / (double)N : 1.0;
    // forward: orders abc, cab, cba; backward: cba, cab, abc
    const int ord[3] = {bwd ? kCba : kAbc, kCab, bwd ? kAbc : kCba};
    const Exchange* ex = bwd ? ds->bwd : ds->fwd;
    void* work = ds->work;
    if (in == work || out == work) return OFFT_ERR_INVALID_ARG;
    // a partial backward flow ends with its data still conjugated
    auto done = [&](int rc) { return rc == OFFT_SUCCESS && bwd && steps < 5 ? conj_in_place(p, out, N, s) : rc; };
    // buffers: each exchange goes from one of out / work to the other (the
    // pack cannot run in place), chosen so that the last step ends in out
    void* b1 = (steps == 1 || steps == 4) ? out : work;   // after step 1
    void* b2 = b1 == work ? out : work;                   // after steps 2 and 3
    void* b3 = b2 == work ? out : work;                   // after step 4
    // step 1: lines of the first order
    int rc = run_lines(p, ord[0], in, b1, bwd, 0, 1.0, s);
    if (rc || steps == 1) return done(rc);
    // step 2: exchange to the middle order
    rc = run_exchange(p, ex[0], method, b1, b2, s);
    if (rc || steps == 2) return done(rc);
    // step 3: lines of the middle order, in place
    rc = run_lines(p, ord[1], b2, b2, 0, 0, 1.0, s);
    if (rc || steps == 3) return done(rc);
    // step 4: exchange to the last order
    rc = run_exchange(p, ex[1], method, b2, b3, s);
    if (rc || steps == 4) return done(rc);
    // step 5: lines of the last order, into out
    return run_lines(p, ord[2], b3, out, 0, bwd, scale, s);
}

// Time of one forward flow with `method` (1 warm-up + reps timed runs,
// minimum of up to two, median of more).
static int time_method(offt_plan_s* p, int method, const void* in, void* out, int reps, hipStream_t s, float* ms) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return OFFT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return OFFT_ERR_HIP; }
    int rc = exec_dist(p, -1, 5, in, out, method, -1, s);
    std::vector<float> runs;
    for (int r = 0; r < reps && rc == OFFT_SUCCESS; ++r) {
        float t = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess) { rc = OFFT_ERR_HIP; break; }
        rc = exec_dist(p, -1, 5, in, out, method, -1, s);
        if (rc) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            rc = OFFT_ERR_HIP;
            break;
        }
        runs.push_back(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::sort(runs.begin(), runs.end());
    if (runs.empty()) *ms = 1e30f;
    else if (runs.size() <= 2) *ms = runs[0];
    else *ms = runs.size() % 2 ? runs[runs.size() / 2] : 0.5f * (runs[runs.size() / 2 - 1] + runs[runs.size() / 2]);
    return rc;
}

static const char* const kMethodName[kDistMethods] = {"Isend_Waitall", "Alltoallv", "Isend_Waitall_Block",
                                                      "Isend_Waitsome", "Isend_Waitsome_Block", "Sendrecv"};

std::string describe_dist(const offt_plan_s* p) {
    const DistState* ds = p->dist;
    char buf[256];
    snprintf(buf, sizeof buf, "dist: %d processes, %s decomposition, method %s, B_SIZE %d", ds->np,
             ds->np <= p->dims[0] && ds->np <= p->dims[2] ? "1-D" : "2-D", kMethodName[ds->method], ds->block);
    std::string out = buf;
    if (ds->method_ms[0] >= 0) {
        out += "; tuned (ms):";
        for (int m = 0; m < kDistMethods; ++m) {
            snprintf(buf, sizeof buf, " %s %.4f", kMethodName[m], ds->method_ms[m]);
            out += buf;
        }
    }
    return out;
}

}  // namespace offt

using namespace offt;

extern "C" {

offt_plan_t offt_plan_dist(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int nprocs, int method, int block_size,
                           const offt_opts* o) {
    offt_opts opts;
    offt_opts_default(&opts);
    if (o) opts = *o;
    int rc = validate_dims(Na, Nb, Nc, dtype, 1);
    const int64_t dims[3] = {Na, Nb, Nc};
    if (rc == OFFT_SUCCESS) {
        // Eq. 2 covers up to N1 N2 processes in every order of the flow
        int64_t lim = kDistMaxProcs;
        for (int ord = 0; ord < 3; ++ord) {
            int64_t n[3];
            order_lengths(dims, ord, n);
            lim = std::min(lim, n[0] * n[1]);
        }
        if (nprocs < 1 || nprocs > lim || method < OFFT_COMM_AUTO || method >= kDistMethods || block_size < 1 ||
            opts.reps < 1)
            rc = OFFT_ERR_INVALID_ARG;
    }
    if (rc != OFFT_SUCCESS) { set_error(rc); return nullptr; }
    rc = check_device();
    if (rc != OFFT_SUCCESS) { set_error(rc); return nullptr; }
    offt_plan_s* p = new offt_plan_s();
    p->kind = 4;
    p->dtype = dtype;
    p->dims[0] = Na; p->dims[1] = Nb; p->dims[2] = Nc;
    p->batch = 1;
    p->normalize = opts.normalize_inverse ? 1 : 0;
    p->dist = new DistState();
    DistState* ds = p->dist;
    ds->np = nprocs;
    ds->block = block_size;
    hipStream_t s = static_cast<hipStream_t>(opts.stream);
    const size_t es = elem_size(dtype);
    const int64_t N = Na * Nb * Nc;
    for (int ord = 0; ord < 3; ++ord) {
        int64_t n[3];
        order_lengths(dims, ord, n);
        dist_line_starts(dims, ord, nprocs, ds->line_start[ord]);
        for (int sp = 0; sp < nprocs; ++sp) {
            PassPlan pp = contiguous_pass(dtype, (int)n[2], ds->line_start[ord][sp + 1] - ds->line_start[ord][sp],
                                          N * (int64_t)es);
            ds->pass[ord][sp] = pp;
            if (n[2] > 1 && rc == OFFT_SUCCESS) {
                if (!pp.k) rc = OFFT_ERR_UNSUPPORTED_SIZE;
                else rc = attach_twiddles(p, &ds->pass[ord][sp], 1, s);
            }
        }
    }
    if (rc == OFFT_SUCCESS) rc = dist_alloc(p, N * es, &ds->work);
    if (rc == OFFT_SUCCESS) rc = dist_alloc(p, N * es, &ds->send);
    if (rc == OFFT_SUCCESS) rc = dist_alloc(p, N * es, &ds->recv);
    if (rc == OFFT_SUCCESS) rc = build_exchange(p, ds, kAbc, kCab, &ds->fwd[0], s);
    if (rc == OFFT_SUCCESS) rc = build_exchange(p, ds, kCab, kCba, &ds->fwd[1], s);
    if (rc == OFFT_SUCCESS) rc = build_exchange(p, ds, kCba, kCab, &ds->bwd[0], s);
    if (rc == OFFT_SUCCESS) rc = build_exchange(p, ds, kCab, kAbc, &ds->bwd[1], s);
    // the communication stream (default priority) and the events of the waits
    if (rc == OFFT_SUCCESS) {
        ds->ev_chunk.assign((size_t)nprocs * nprocs, nullptr);
        if (hipStreamCreateWithFlags(&ds->comm, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ds->ev_start, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ds->ev_group, hipEventDisableTiming) != hipSuccess)
            rc = OFFT_ERR_HIP;
        for (size_t i = 0; i < ds->ev_chunk.size() && rc == OFFT_SUCCESS; ++i)
            if (hipEventCreateWithFlags(&ds->ev_chunk[i], hipEventDisableTiming) != hipSuccess) rc = OFFT_ERR_HIP;
    }
    if (rc == OFFT_SUCCESS && hipStreamSynchronize(s) != hipSuccess) rc = OFFT_ERR_HIP;
    // the method: given (User-select), or every one timed here (auto-tuning
    // in the initialization phase, Sec. 3.2.3); ties keep the lower id
    if (rc == OFFT_SUCCESS && method == OFFT_COMM_AUTO) {
        void *tin = nullptr, *tout = nullptr;
        if (hipMalloc(&tin, N * es) != hipSuccess || hipMalloc(&tout, N * es) != hipSuccess) {
            (void)hipGetLastError();
            rc = OFFT_ERR_OUT_OF_MEMORY;
        }
        if (rc == OFFT_SUCCESS && launch_fill_uniform(tin, N, dtype, 1501, s) != hipSuccess) rc = OFFT_ERR_HIP;
        float best = 1e30f;
        int best_m = OFFT_COMM_ISEND_WAITSOME;
        for (int m = 0; m < kDistMethods && rc == OFFT_SUCCESS; ++m) {
            float ms = 0.f;
            rc = time_method(p, m, tin, tout, opts.reps, s, &ms);
            ds->method_ms[m] = ms;
            if (rc == OFFT_SUCCESS && ms < best) { best = ms; best_m = m; }
        }
        (void)hipStreamSynchronize(s);
        if (tin) (void)hipFree(tin);
        if (tout) (void)hipFree(tout);
        ds->method = best_m;
    } else if (rc == OFFT_SUCCESS) {
        ds->method = method;
    }
    if (rc != OFFT_SUCCESS) { free_plan(p); set_error(rc); return nullptr; }
    set_error(OFFT_SUCCESS);
    return p;
}

int offt_dist_method(offt_plan_t p) {
    if (!p) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    if (p->kind != 4 || !p->dist) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    set_error(OFFT_SUCCESS);
    return p->dist->method;
}

int offt_dist_method_times(offt_plan_t p, float* ms) {
    if (!p || !ms) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    if (p->kind != 4 || !p->dist) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    for (int m = 0; m < kDistMethods; ++m) ms[m] = p->dist->method_ms[m];
    set_error(OFFT_SUCCESS);
    return kDistMethods;
}

int64_t offt_dist_count(offt_plan_t p, int direction, int step, int src, int dst) {
    if (!p || (direction != OFFT_FORWARD && direction != OFFT_BACKWARD) || step < 0 || step > 1) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    if (p->kind != 4 || !p->dist) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    const DistState* ds = p->dist;
    if (src < 0 || src >= ds->np || dst < 0 || dst >= ds->np) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    const Exchange& ex = direction == OFFT_FORWARD ? ds->fwd[step] : ds->bwd[step];
    set_error(OFFT_SUCCESS);
    return ex.count[(size_t)src * ds->np + dst];
}

int64_t offt_dist_block(offt_plan_t p, int order, int proc, int64_t* end) {
    if (!p || order < 0 || order > 2) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    if (p->kind != 4 || !p->dist) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    const DistState* ds = p->dist;
    if (proc < 0 || proc >= ds->np) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    int64_t n[3];
    order_lengths(p->dims, order, n);
    if (end) *end = ds->line_start[order][proc + 1] * n[2];
    set_error(OFFT_SUCCESS);
    return ds->line_start[order][proc] * n[2];
}

int offt_dist_exec_steps(offt_plan_t p, int direction, int steps, int method, const void* in, void* out,
                         void* stream) {
    if (!p || !in || !out || (direction != OFFT_FORWARD && direction != OFFT_BACKWARD) || steps < 1 || steps > 5 ||
        method < OFFT_COMM_AUTO || method >= kDistMethods) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    if (p->kind != 4 || !p->dist) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    const int rc = exec_dist(p, direction, steps, in, out, method, -1, static_cast<hipStream_t>(stream));
    set_error(rc);
    return rc;
}

}  // extern "C"
