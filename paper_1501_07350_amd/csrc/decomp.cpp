// decomp.cpp -- byte and volume accounting (host only, no device).
//
// Per plan: the HBM bytes one axis pass moves.  Per decomposition: the
// paper's row-wise block distribution (Sec. 2, Eq. 2 and the ranges derived
// from it) and the number of elements each transpose of the abc -> cab -> cba
// sequence (Fig. 1b) moves from one process to another, the quantity whose
// total the paper plots as the volume of communication (Sec. 4.1).  On one
// GPU nothing is exchanged; these counts describe how the transform would
// shard over several.
#include <algorithm>
#include <cstdint>

#include "../../include/offt.h"
#include "offt_internal.h"
#include "plan_impl.h"

namespace offt {

// f(N1, N2, N3, Np, id) of Eq. 2: first linear index of process id's block.
// Whole N2 x N3 planes when Np <= N1, whole N3-lines when N1 < Np <= N1 N2.
static int64_t block_start(int64_t n1, int64_t n2, int64_t n3, int64_t np, int64_t id) {
    if (np <= n1) return (n1 * id / np) * n2 * n3;
    return (n1 * n2 * id / np) * n3;
}

// Number of integers k in [0, n) with lo <= k*m + r < hi (m > 0).
static int64_t count_progression(int64_t n, int64_t m, int64_t r, int64_t lo, int64_t hi) {
    auto ceil_div = [](int64_t x, int64_t d) { return x >= 0 ? (x + d - 1) / d : -((-x) / d); };
    const int64_t k0 = std::max<int64_t>(0, ceil_div(lo - r, m));
    const int64_t k1 = std::min<int64_t>(n, ceil_div(hi - r, m));
    return std::max<int64_t>(0, k1 - k0);
}

// Elements process src holds before transpose `step` and process dst after
// it (step 0: abc -> cab, step 1: cab -> cba).
static int64_t transpose_count(int64_t n1, int64_t n2, int64_t n3, int64_t np, int step, int64_t src,
                               int64_t dst) {
    int64_t total = 0;
    if (step == 0) {
        // abc blocks are whole c-lines: pairs ab = a*n2 + b in [p0, p1);
        // cab blocks (order c, a, b) are whole b-lines: pairs c*n1 + a in [q0, q1)
        const int64_t p0 = block_start(n1, n2, n3, np, src) / n3, p1 = block_start(n1, n2, n3, np, src + 1) / n3;
        const int64_t q0 = block_start(n3, n1, n2, np, dst) / n2, q1 = block_start(n3, n1, n2, np, dst + 1) / n2;
        if (p0 >= p1 || q0 >= q1) return 0;
        for (int64_t a = p0 / n2; a <= (p1 - 1) / n2; ++a) {
            const int64_t nb = std::min(p1, a * n2 + n2) - std::max(p0, a * n2);
            total += nb * count_progression(n3, n1, a, q0, q1);
        }
    } else {
        // cab blocks: pairs c*n1 + a in [p0, p1); cba blocks (order c, b, a)
        // are whole a-lines: pairs c*n2 + b in [q0, q1)
        const int64_t p0 = block_start(n3, n1, n2, np, src) / n2, p1 = block_start(n3, n1, n2, np, src + 1) / n2;
        const int64_t q0 = block_start(n3, n2, n1, np, dst) / n1, q1 = block_start(n3, n2, n1, np, dst + 1) / n1;
        if (p0 >= p1 || q0 >= q1) return 0;
        const int64_t c_lo = std::max(p0 / n1, q0 / n2), c_hi = std::min((p1 - 1) / n1, (q1 - 1) / n2);
        for (int64_t c = c_lo; c <= c_hi; ++c) {
            const int64_t na = std::min(p1, c * n1 + n1) - std::max(p0, c * n1);
            const int64_t nb = std::min(q1, c * n2 + n2) - std::max(q0, c * n2);
            if (na > 0 && nb > 0) total += na * nb;
        }
    }
    return total;
}

// Eq. 2 covers Np <= N1 N2 of the order being decomposed; both orders of a
// transpose must qualify.
static bool decomp_ok(int64_t n1, int64_t n2, int64_t n3, int64_t np, int step) {
    if (n1 < 1 || n2 < 1 || n3 < 1 || np < 1 || (step != 0 && step != 1)) return false;
    if (n1 > (int64_t(1) << 20) || n2 > (int64_t(1) << 20) || n3 > (int64_t(1) << 20)) return false;
    if (step == 0) return np <= n1 * n2 && np <= n3 * n1;
    return np <= n3 * n1 && np <= n3 * n2;
}

}  // namespace offt

using namespace offt;

extern "C" {

int64_t offt_decomp_start(int64_t n1, int64_t n2, int64_t n3, int64_t np, int64_t id) {
    if (n1 < 1 || n2 < 1 || n3 < 1 || np < 1 || np > n1 * n2 || id < 0 || id > np ||
        n1 > (int64_t(1) << 20) || n2 > (int64_t(1) << 20) || n3 > (int64_t(1) << 20)) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    set_error(OFFT_SUCCESS);
    return block_start(n1, n2, n3, np, id);
}

int64_t offt_transpose_count(int64_t n1, int64_t n2, int64_t n3, int64_t np, int step, int64_t src,
                             int64_t dst) {
    if (!decomp_ok(n1, n2, n3, np, step) || src < 0 || src >= np || dst < 0 || dst >= np) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    set_error(OFFT_SUCCESS);
    return transpose_count(n1, n2, n3, np, step, src, dst);
}

int64_t offt_transpose_volume(int64_t n1, int64_t n2, int64_t n3, int64_t np, int step) {
    if (!decomp_ok(n1, n2, n3, np, step)) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    int64_t moved = 0;
    for (int64_t p = 0; p < np; ++p) {
        const int64_t held = step == 0 ? block_start(n1, n2, n3, np, p + 1) - block_start(n1, n2, n3, np, p)
                                       : block_start(n3, n1, n2, np, p + 1) - block_start(n3, n1, n2, np, p);
        moved += held - transpose_count(n1, n2, n3, np, step, p, p);
    }
    set_error(OFFT_SUCCESS);
    return moved;
}

int64_t offt_pass_bytes(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch) {
    const int rc = validate_dims(Na, Nb, Nc, dtype, batch);
    if (rc != OFFT_SUCCESS) {
        set_error(rc);
        return rc;
    }
    set_error(OFFT_SUCCESS);
    // one read and one write of every element; the twiddle table (L values
    // per tile, served from cache after the first tiles) is not counted
    return 2 * Na * Nb * Nc * batch * (int64_t)elem_size(dtype);
}

}  // extern "C"
