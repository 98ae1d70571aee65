// dist_device.hpp -- device code of the exchanges of the distributed flow
// (dist.hip): pack, unpack and the chunk copies.
//
// One exchange (O_in -> O_out) moves each element of process src to the
// process dst that owns its linear index in O_out (Duy & Ozaki, Sec. 2 and
// Sec. 3.1.1: pack, communicate, unpack).  Each of the flow's exchanges is a
// transpose of the global array, so one of pack and unpack has to move data
// across the fastest axis: here the pack does it, through LDS tiles, and
// the unpack copies contiguous runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace offt {

constexpr int kPackThreads = 256;    // pack: a 32 x 32 tile, 8 rows of threads
constexpr int kPackTile = 32;
constexpr int kGatherThreads = 256;  // unpack: one wavefront per line
constexpr int kCopyThreads = 256;

// Chunk (src, dst) holds the elements src sends dst in dst's O_out order, so
// that the unpack copies whole runs.  Along an O_out line (its fastest axis,
// k') the O_in line index is base + k' * step, increasing, so the elements
// of one O_out line that come from one process form one run; the tables of
// the reverse exchange O_out -> O_in (klo, cnt, pre: that run per process
// and line coordinate q, and prefix sums over q) give every element's place
// in its chunk in closed form.
struct ReverseTables {
    const int64_t* klo;        // [proc * nq + q]: first k' of the run process proc owns on a line with coordinate q
    const int64_t* cnt;        // [proc * nq + q]: its length
    const int64_t* pre;        // [proc * (nq + 1) + q]: sum of cnt over q' < q
    const int64_t* in_start;   // [np + 1]: first O_in line of each process
    int64_t nm;                // middle length of O_out
    int64_t base_mul, step;    // O_in line of element k' of O_out line m: base_mul * q(m) + step * k'
    int nq;                    // values of q
    int q_slowest;             // q = m / nm (1) or m % nm (0)
};

// Line indices and lengths fit 32 bits (axes of at most 1024 points: at
// most 2^20 lines), so the divisions by the middle length are 32-bit ones.
__device__ __forceinline__ int64_t rev_q(const ReverseTables& t, int64_t m) {
    const uint32_t mm = (uint32_t)m, nm = (uint32_t)t.nm;
    return t.q_slowest ? mm / nm : mm % nm;
}

// Elements of the O_out lines [0, m) that come from process proc (the
// process that owns them in O_in).
__device__ __forceinline__ int64_t rev_prefix(const ReverseTables& t, int proc, int64_t m) {
    const int64_t* pre = t.pre + (int64_t)proc * (t.nq + 1);
    const uint32_t mm = (uint32_t)m, nm = (uint32_t)t.nm;
    const uint32_t q = mm / nm, r = mm - q * nm;
    if (t.q_slowest) return t.nm * pre[q] + (int64_t)r * ((int)q < t.nq ? t.cnt[(int64_t)proc * t.nq + q] : 0);
    return (int64_t)q * pre[t.nq] + pre[r];
}

__device__ __forceinline__ int dist_owner(const int64_t* start, int np, int64_t line) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= line) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Pack of process src: its O_in lines [line_begin, line_end), read as tiles
// of 32 values of the O_in coordinate u that is O_out's fastest axis (the
// middle or the slowest O_in axis) by 32 values of k (O_in's fastest axis)
// at one value of the remaining coordinate v; transposed through LDS and
// written along u into the chunks.  Reads and writes run along 32
// consecutive elements.
struct PackArgs {
    const void* from;          // the global O_in array
    void* send;                // chunks to other processes: send + sdispl[src * np + dst]
    void* self;                // src's own chunk (the receive array at its place, or the O_out array itself)
    const int64_t* sdispl;     // [src * np + dst]
    const int64_t* out_start;  // [np + 1]: first O_out line of each process
    ReverseTables rev;
    int64_t in_n[3];           // O_in lengths, slowest first
    int64_t out_n[3];
    int in_ax[3], out_ax[3];
    int64_t line_begin, line_end;
    int64_t v_lo, v_n;         // v range of the tiles
    int64_t u_lo, u_n;         // u range of the tiles
    int64_t u_tiles, k_tiles;  // tiles along u and k
    int u_slowest;             // u is O_in's slowest (1) or middle (0) axis
    int np, src;
};

// LDS of one pack tile: the elements, and per tile column (one k) the place
// of its first element's run in the chunk it goes to.
template <typename V>
struct PackShared {
    V tile[kPackTile][kPackTile + 1];
    int64_t col_off[kPackTile];   // element offset of u = 0 in the column's destination array
    int col_self[kPackTile];      // the column goes to src's own chunk
};

template <typename V>
__device__ __forceinline__ void pack_tile(const PackArgs& a, PackShared<V>& sh) {
    const V* __restrict__ from = static_cast<const V*>(a.from);
    const int64_t nm = a.in_n[1], nf = a.in_n[2];
    const int64_t b = blockIdx.x;
    const int64_t kt = b % a.k_tiles;
    const int64_t ut = (b / a.k_tiles) % a.u_tiles;
    const int64_t v = a.v_lo + b / (a.k_tiles * a.u_tiles);
    const int64_t u0 = a.u_lo + ut * kPackTile, k0 = kt * kPackTile;
    const int lane = (int)(threadIdx.x % kPackTile), row = (int)(threadIdx.x / kPackTile);
    constexpr int kRows = kPackThreads / kPackTile;
    // read: row r of the tile is line (u0 + r, v), lanes along k
    for (int r = row; r < kPackTile; r += kRows) {
        const int64_t u = u0 + r, k = k0 + lane;
        const int64_t l = a.u_slowest ? u * nm + v : v * nm + u;
        if (u < a.u_lo + a.u_n && k < nf && l >= a.line_begin && l < a.line_end) sh.tile[r][lane] = from[l * nf + k];
    }
    // meanwhile, the first wavefront places the tile's columns: column k
    // lies on one O_out line m (u is O_out's fastest axis), owned by d
    if (threadIdx.x < kPackTile && k0 + threadIdx.x < nf) {
        int64_t co[3];
        co[a.in_ax[a.u_slowest ? 1 : 0]] = v;
        co[a.in_ax[2]] = k0 + threadIdx.x;
        co[a.in_ax[a.u_slowest ? 0 : 1]] = 0;
        const int64_t m = co[a.out_ax[0]] * a.out_n[1] + co[a.out_ax[1]];
        const int d = dist_owner(a.out_start, a.np, m);
        const int64_t q = rev_q(a.rev, m);
        const int64_t pos0 = rev_prefix(a.rev, a.src, m) - rev_prefix(a.rev, a.src, a.out_start[d]) -
                             a.rev.klo[(int64_t)a.src * a.rev.nq + q];
        sh.col_self[threadIdx.x] = d == a.src;
        sh.col_off[threadIdx.x] = d == a.src ? pos0 : a.sdispl[a.src * a.np + d] + pos0;
    }
    __syncthreads();
    // write: column c of the tile is k = k0 + c, lanes along u (O_out's k')
    const int64_t u = u0 + lane;
    const int64_t l = a.u_slowest ? u * nm + v : v * nm + u;
    if (u >= a.u_lo + a.u_n || l < a.line_begin || l >= a.line_end) return;
    for (int c = row; c < kPackTile && k0 + c < nf; c += kRows) {
        V* __restrict__ dst = sh.col_self[c] ? static_cast<V*>(a.self) : static_cast<V*>(a.send);
        dst[sh.col_off[c] + u] = sh.tile[lane][c];
    }
}

// Unpack of process dst: its O_out lines [line_begin, line_end), one
// wavefront per line; the runs of the line come from the processes that own
// its O_in lines, each a contiguous piece of that process's chunk in the
// receive array.  src_only >= 0 unpacks that process's chunk only.
struct GatherArgs {
    const void* recv;          // receive array: recv + rdispl[dst * np + src] is chunk (src, dst)
    void* to;                  // the global O_out array
    const int64_t* rdispl;     // [dst * np + src]
    ReverseTables rev;
    int64_t nf;                // O_out's fastest length
    int64_t line_begin, line_end;
    int np, dst, src_only;
    int pad_;
};

template <typename V>
__device__ __forceinline__ void gather_lines(const GatherArgs& a) {
    const V* __restrict__ recv = static_cast<const V*>(a.recv);
    V* __restrict__ to = static_cast<V*>(a.to);
    const int lane = (int)(threadIdx.x % 64);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t m = a.line_begin + (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; m < a.line_end;
         m += waves) {
        const int64_t q = rev_q(a.rev, m);
        const int64_t base = a.rev.base_mul * q;
        int s0 = dist_owner(a.rev.in_start, a.np, base);
        int s1 = dist_owner(a.rev.in_start, a.np, base + a.rev.step * (a.nf - 1));
        if (a.src_only >= 0) {
            if (a.src_only < s0 || a.src_only > s1) continue;
            s0 = s1 = a.src_only;
        }
        for (int s = s0; s <= s1; ++s) {
            const int64_t c = a.rev.cnt[(int64_t)s * a.rev.nq + q];
            if (c == 0) continue;
            const int64_t k0 = a.rev.klo[(int64_t)s * a.rev.nq + q];
            const V* __restrict__ src = recv + a.rdispl[(int64_t)a.dst * a.np + s] + rev_prefix(a.rev, s, m) -
                                        rev_prefix(a.rev, s, a.line_begin);
            V* __restrict__ dst = to + m * a.nf + k0;
            for (int64_t j = lane; j < c; j += 64) dst[j] = src[j];
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
