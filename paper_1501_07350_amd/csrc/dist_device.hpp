// dist_device.hpp -- device code of the exchanges of the distributed flow
// (dist.hip): pack, unpack and the chunk copies.
//
// One exchange (O_in -> O_out) moves each element of process src to the
// process dst that owns its linear index in O_out (Duy & Ozaki, Sec. 2 and
// Sec. 3.1.1: pack, communicate, unpack).  Along a line of O_in (its fastest
// axis, k) the O_out line index is base + k*step, increasing, so the
// elements of one line that go to one dst form one run [klo, klo + cnt);
// base depends on one coordinate q of the line (its slowest or its middle
// coordinate), so the number of elements dst receives from the lines before
// line l is a closed form over per-q counts and their prefix sums
// (route_prefix).  Chunk (src, dst) holds those elements in src's order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace offt {

constexpr int kRouteThreads = 256;
constexpr int kCopyThreads = 256;

struct RouteArgs {
    const void* from;          // pack: global O_in array; unpack: receive array
    void* to;                  // pack: send array; unpack: global O_out array
    const int64_t* sdispl;     // [src * np + dst]: chunk (src, dst) in the send array
    const int64_t* rdispl;     // [dst * np + src]: chunk (src, dst) in the receive array
    const int64_t* klo;        // [dst * nq + q]: first k of the run of a line with coordinate q
    const int64_t* cnt;        // [dst * nq + q]: length of that run
    const int64_t* pre;        // [dst * (nq + 1) + q]: sum of cnt over q' < q
    const int64_t* out_start;  // [np + 1]: first O_out line of each process
    int64_t in_n[3];           // O_in lengths, slowest first
    int64_t out_n[3];          // O_out lengths
    int in_ax[3], out_ax[3];   // axes of O_in / O_out, slowest first
    int64_t line_begin, line_end;   // O_in lines of the source process
    int64_t base_mul, step;    // O_out line = base_mul * q + step * k
    int nq;                    // values of q
    int q_slowest;             // q = l / n_m (1) or l % n_m (0)
    int src;                   // source process
    int dst_only;              // one destination process, or -1 for all
    int np;
    int unpack;
};

__device__ __forceinline__ int64_t route_prefix(const RouteArgs& r, int d, int64_t l) {
    const int64_t nm = r.in_n[1];
    const int64_t* pre = r.pre + (int64_t)d * (r.nq + 1);
    if (r.q_slowest) {
        const int64_t q = l / nm;
        return nm * pre[q] + (l - q * nm) * r.cnt[(int64_t)d * r.nq + q];
    }
    const int64_t q = l % nm;
    return (l / nm) * pre[r.nq] + pre[q];
}

__device__ __forceinline__ int route_owner(const int64_t* start, int np, int64_t line) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= line) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Linear index in O_out of the element (l, k) of O_in.
__device__ __forceinline__ int64_t route_out_index(const RouteArgs& r, int64_t l, int64_t k) {
    int64_t co[3];
    co[r.in_ax[0]] = l / r.in_n[1];
    co[r.in_ax[1]] = l % r.in_n[1];
    co[r.in_ax[2]] = k;
    return (co[r.out_ax[0]] * r.out_n[1] + co[r.out_ax[1]]) * r.out_n[2] + co[r.out_ax[2]];
}

// Pack or unpack of the source process's lines, one line per workgroup
// (grid-stride over blockIdx.x).  Pack reads the line in order and writes each run to its
// chunk; unpack reads the runs from the receive array and writes each element
// to its O_out place.
template <typename V>
__device__ __forceinline__ void route_lines(const RouteArgs& r) {
    const V* __restrict__ from = static_cast<const V*>(r.from);
    V* __restrict__ to = static_cast<V*>(r.to);
    const int64_t nf = r.in_n[2];
    for (int64_t l = r.line_begin + blockIdx.x; l < r.line_end; l += gridDim.x) {
        const int64_t q = r.q_slowest ? l / r.in_n[1] : l % r.in_n[1];
        const int64_t base = r.base_mul * q;
        if (r.dst_only >= 0) {
            const int d = r.dst_only;
            const int64_t c = r.cnt[(int64_t)d * r.nq + q];
            if (c == 0) continue;
            const int64_t k0 = r.klo[(int64_t)d * r.nq + q];
            const int64_t pos0 = route_prefix(r, d, l) - route_prefix(r, d, r.line_begin);
            for (int64_t j = threadIdx.x; j < c; j += blockDim.x) {
                if (r.unpack)
                    to[route_out_index(r, l, k0 + j)] = from[r.rdispl[(int64_t)d * r.np + r.src] + pos0 + j];
                else
                    to[r.sdispl[(int64_t)r.src * r.np + d] + pos0 + j] = from[l * nf + k0 + j];
            }
            continue;
        }
        for (int64_t k = threadIdx.x; k < nf; k += blockDim.x) {
            const int d = route_owner(r.out_start, r.np, base + r.step * k);
            const int64_t pos = route_prefix(r, d, l) - route_prefix(r, d, r.line_begin) +
                                (k - r.klo[(int64_t)d * r.nq + q]);
            if (r.unpack)
                to[route_out_index(r, l, k)] = from[r.rdispl[(int64_t)d * r.np + r.src] + pos];
            else
                to[r.sdispl[(int64_t)r.src * r.np + d] + pos] = from[l * nf + k];
        }
    }
}

// Communication: copies of chunks (send -> receive), one descriptor per
// chunk; blockIdx.y picks the descriptor.
struct CopyDesc {
    int64_t from, to, n;
};

template <typename V>
__device__ __forceinline__ void copy_chunk(const V* __restrict__ send, V* __restrict__ recv, const CopyDesc& d) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.n; i += (int64_t)gridDim.x * blockDim.x)
        recv[d.to + i] = send[d.from + i];
}

}  // namespace offt
