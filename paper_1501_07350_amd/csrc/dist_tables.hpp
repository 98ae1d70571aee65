// dist_tables.hpp -- host-side tables of the distributed flow (dist.hip):
// the Eq. 2 blocks of every order and, per exchange, the runs each line of a
// process sends each other process, the chunk sizes and their places in the
// send and receive arrays.  Plain C++ (no HIP): the library builds its
// exchanges with it, and the CPU emulation of the exchange kernels uses the
// same tables.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace offt {

// axes of the three orders, slowest first (a = 0, b = 1, c = 2)
constexpr int kOrderAxes[3][3] = {{0, 1, 2}, {2, 0, 1}, {2, 1, 0}};
enum { kAbc = 0, kCab = 1, kCba = 2 };

inline void order_lengths(const int64_t dims[3], int order, int64_t n[3]) {
    for (int i = 0; i < 3; ++i) n[i] = dims[kOrderAxes[order][i]];
}

// f(N1, N2, N3, Np, id) of Eq. 2: first linear index of process id's block
inline int64_t eq2_start(int64_t n1, int64_t n2, int64_t n3, int64_t np, int64_t id) {
    if (np <= n1) return (n1 * id / np) * n2 * n3;
    return (n1 * n2 * id / np) * n3;
}

// First line (of the order's fastest axis) of every process, np + 1 values.
inline void dist_line_starts(const int64_t dims[3], int order, int np, int64_t* starts) {
    int64_t n[3];
    order_lengths(dims, order, n);
    for (int q = 0; q <= np; ++q) starts[q] = eq2_start(n[0], n[1], n[2], np, q) / n[2];
}

struct ExchangeTables {
    int64_t in_n[3], out_n[3];        // lengths of O_in and O_out, slowest first
    int in_ax[3], out_ax[3];          // their axes
    int64_t base_mul = 0, step = 0;   // O_out line of element (l, k) of O_in: base_mul * q(l) + step * k
    int nq = 0;                       // values of q
    int q_slowest = 0;                // q = l / n_m (1) or l % n_m (0), n_m the middle length of O_in
    std::vector<int64_t> klo, cnt;    // [dst * nq + q]: the run a line with coordinate q sends dst
    std::vector<int64_t> pre;         // [dst * (nq + 1) + q]: sum of cnt over q' < q
    std::vector<int64_t> count;       // [src * np + dst]: chunk sizes
    std::vector<int64_t> sdispl;      // [src * np + dst]: chunk offsets in the send array
    std::vector<int64_t> rdispl;      // [dst * np + src]: chunk offsets in the receive array
    int64_t max_chunk = 0;

    // Elements dst receives from the O_in lines [0, l).
    int64_t prefix(int d, int64_t l) const {
        const int64_t nm = in_n[1];
        const int64_t* pr = pre.data() + (size_t)d * (nq + 1);
        if (q_slowest) {
            const int64_t q = l / nm;
            return nm * pr[q] + (l - q * nm) * (q < nq ? cnt[(size_t)d * nq + q] : 0);
        }
        return (l / nm) * pr[nq] + pr[l % nm];
    }
};

// Tables of the exchange in_order -> out_order over np processes whose O_in
// and O_out lines start at in_start / out_start (np + 1 values each).
// Returns false if the two orders are not one of the flow's transposes (the
// fastest axis of O_in must be the slowest or the middle axis of O_out) or
// the chunks do not tile the processes' slices.
inline bool build_exchange_tables(const int64_t dims[3], int np, int in_order, int out_order,
                                  const int64_t* in_start, const int64_t* out_start, ExchangeTables* t) {
    order_lengths(dims, in_order, t->in_n);
    order_lengths(dims, out_order, t->out_n);
    for (int i = 0; i < 3; ++i) {
        t->in_ax[i] = kOrderAxes[in_order][i];
        t->out_ax[i] = kOrderAxes[out_order][i];
    }
    // the fastest axis f of O_in is the slowest or the middle axis of O_out;
    // the other of those two, u, is the coordinate the O_out line base
    // depends on, and it is the slowest or the middle axis of O_in
    const int f = t->in_ax[2];
    if (t->out_ax[0] != f && t->out_ax[1] != f) return false;
    const int u = t->out_ax[0] == f ? t->out_ax[1] : t->out_ax[0];
    t->step = t->out_ax[0] == f ? t->out_n[1] : 1;
    t->base_mul = t->out_ax[0] == u ? t->out_n[1] : 1;
    t->q_slowest = t->in_ax[0] == u ? 1 : 0;
    t->nq = (int)(t->q_slowest ? t->in_n[0] : t->in_n[1]);
    const int nq = t->nq;
    const int64_t nf = t->in_n[2];
    t->klo.assign((size_t)np * nq, 0);
    t->cnt.assign((size_t)np * nq, 0);
    t->pre.assign((size_t)np * (nq + 1), 0);
    for (int d = 0; d < np; ++d) {
        const int64_t Ls = out_start[d], Le = out_start[d + 1];   // O_out lines of d: [Ls, Le)
        int64_t acc = 0;
        for (int q = 0; q < nq; ++q) {
            const int64_t base = t->base_mul * q;
            // k with Ls <= base + step * k < Le and 0 <= k < nf
            int64_t lo = Ls <= base ? 0 : (Ls - base + t->step - 1) / t->step;
            int64_t hi = Le - 1 < base ? -1 : (Le - 1 - base) / t->step;
            hi = std::min<int64_t>(hi, nf - 1);
            const int64_t c = hi >= lo ? hi - lo + 1 : 0;
            t->klo[(size_t)d * nq + q] = c ? lo : 0;
            t->cnt[(size_t)d * nq + q] = c;
            t->pre[(size_t)d * (nq + 1) + q] = acc;
            acc += c;
        }
        t->pre[(size_t)d * (nq + 1) + nq] = acc;
    }
    t->count.assign((size_t)np * np, 0);
    for (int sp = 0; sp < np; ++sp)
        for (int d = 0; d < np; ++d)
            t->count[(size_t)sp * np + d] = t->prefix(d, in_start[sp + 1]) - t->prefix(d, in_start[sp]);
    // send: src's slice of the O_in array, chunks by dst; receive: dst's
    // slice of the O_out array, chunks by src
    t->sdispl.assign((size_t)np * np, 0);
    t->rdispl.assign((size_t)np * np, 0);
    t->max_chunk = 0;
    for (int sp = 0; sp < np; ++sp) {
        int64_t off = in_start[sp] * nf;
        for (int d = 0; d < np; ++d) {
            t->sdispl[(size_t)sp * np + d] = off;
            off += t->count[(size_t)sp * np + d];
            t->max_chunk = std::max(t->max_chunk, t->count[(size_t)sp * np + d]);
        }
        if (off != in_start[sp + 1] * nf) return false;
    }
    for (int d = 0; d < np; ++d) {
        int64_t off = out_start[d] * t->out_n[2];
        for (int sp = 0; sp < np; ++sp) {
            t->rdispl[(size_t)d * np + sp] = off;
            off += t->count[(size_t)sp * np + d];
        }
        if (off != out_start[d + 1] * t->out_n[2]) return false;
    }
    return true;
}

}  // namespace offt
