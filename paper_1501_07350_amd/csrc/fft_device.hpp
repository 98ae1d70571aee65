// fft_device.hpp -- device code of one axis pass of the 3-D transform.
//
// One axis pass applies a length-L 1-D DFT to every "line" of a [M1][L][M2]
// view of the data (the paper's step "transform in a particular dimension",
// Sec. 3.1.1).  With the grid stored row-major (Sec. 2, Eq. 1):
//   c axis: M1 = batch*Na*Nb, M2 = 1          (lines contiguous)
//   b axis: M1 = batch*Na,    M2 = Nc         (lines strided by Nc)
//   a axis: M1 = batch,       M2 = Nb*Nc      (lines strided by Nb*Nc)
// A workgroup owns W lines.  It stages them from HBM into LDS with coalesced
// accesses (W consecutive columns per row for strided lines: this is where
// the paper's pack/transpose step happens on one GPU), runs the radix stages
// out of LDS, and writes the tile back the same way.  Each pass reads and
// writes the grid exactly once.
//
// The 1-D DFT is a Stockham autosort FFT: stage s with radix R and span Ns
// (product of the previous radices) takes butterfly b in [0, L/R), reads
// x[b + r*L/R] for r < R, multiplies element r by W_{Ns R}^(r (b mod Ns)),
// applies the R-point DFT and writes element r to
// (b div Ns)*Ns*R + (b mod Ns) + r*Ns.  After the last stage the result is in
// natural order.  Only forward butterflies exist: the backward transform is
// conj(F(conj(x))), folded into the first load and the last store.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace offt {

template <typename S> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
// multiply by -i
template <typename V> __device__ __forceinline__ V mul_mi(V a) { V r; r.x = a.y; r.y = -a.x; return r; }
// multiply by +i
template <typename V> __device__ __forceinline__ V mul_pi(V a) { V r; r.x = -a.y; r.y = a.x; return r; }
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { V r; r.x = a.x * s; r.y = a.y * s; return r; }

// ---- small forward DFTs on registers (W_R = exp(-2 pi i / R)) -----------------
// Each is derived from the definition y_k = sum_j x_j W_R^(jk) by pairing
// x_j with x_{R-j} (radix 3, 5) or by one even/odd split (radix 4, 8, 16, 32).

template <typename V> __device__ __forceinline__ void dft2(V& a, V& b) {
    V t = a; a = cadd(t, b); b = csub(t, b);
}

template <typename V> __device__ __forceinline__ void dft3(V* v) {
    using S = decltype(v[0].x);
    const S c = S(-0.5);                                   // cos(2pi/3)
    const S s = S(-0.86602540378443864676372317075294);    // -sin(2pi/3)
    V a = cadd(v[1], v[2]);
    V d = csub(v[1], v[2]);
    V t = cadd(v[0], cscale(a, c));
    V u = cscale(d, s);          // y1 = t + i u, y2 = t - i u
    v[0] = cadd(v[0], a);
    v[1] = cadd(t, mul_pi(u));
    v[2] = csub(t, mul_pi(u));
}

template <typename V> __device__ __forceinline__ void dft4(V* v) {
    V s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    V s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, mul_mi(d13));
    v[3] = csub(d02, mul_mi(d13));
}

template <typename V> __device__ __forceinline__ void dft5(V* v) {
    using S = decltype(v[0].x);
    const S c1 = S(0.30901699437494742410229341718282);    // cos(2pi/5)
    const S c2 = S(-0.80901699437494742410229341718282);   // cos(4pi/5)
    const S s1 = S(-0.95105651629515357211643933337938);   // -sin(2pi/5)
    const S s2 = S(-0.58778525229247312916870595463907);   // -sin(4pi/5)
    V a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    V a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    V t1 = cadd(v[0], cadd(cscale(a1, c1), cscale(a2, c2)));
    V t2 = cadd(v[0], cadd(cscale(a1, c2), cscale(a2, c1)));
    V u1 = cadd(cscale(b1, s1), cscale(b2, s2));   // y1 = t1 + i u1, y4 = t1 - i u1
    V u2 = csub(cscale(b1, s2), cscale(b2, s1));   // y2 = t2 + i u2, y3 = t2 - i u2
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(t1, mul_pi(u1));
    v[4] = csub(t1, mul_pi(u1));
    v[2] = cadd(t2, mul_pi(u2));
    v[3] = csub(t2, mul_pi(u2));
}

// y_k = E_k + W_8^k O_k, y_{k+4} = E_k - W_8^k O_k with E, O the 4-point DFTs
// of the even and odd samples.
template <typename V> __device__ __forceinline__ void dft8(V* v) {
    using S = decltype(v[0].x);
    const S h = S(0.70710678118654752440084436210485);     // sqrt(2)/2
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    dft4(e);
    dft4(o);
    V o1; o1.x = h * (o[1].x + o[1].y); o1.y = h * (o[1].y - o[1].x);     // W8^1 = h(1 - i)
    V o2 = mul_mi(o[2]);                                                // W8^2 = -i
    V o3; o3.x = h * (o[3].y - o[3].x); o3.y = -h * (o[3].x + o[3].y);  // W8^3 = h(-1 - i)
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
}

template <typename V> __device__ __forceinline__ void dft16(V* v) {
    using S = decltype(v[0].x);
    // W16^k = cos(k pi/8) - i sin(k pi/8), k = 1..7
    const S c1 = S(0.92387953251128675612818318939679);
    const S s1 = S(0.38268343236508977172845998403040);
    const S h = S(0.70710678118654752440084436210485);
    V e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { e[k] = v[2 * k]; o[k] = v[2 * k + 1]; }
    dft8(e);
    dft8(o);
    V w[8];
    w[0] = o[0];
    { V t; t.x = c1 * o[1].x + s1 * o[1].y; t.y = c1 * o[1].y - s1 * o[1].x; w[1] = t; }   // (c1 - i s1)
    { V t; t.x = h * (o[2].x + o[2].y); t.y = h * (o[2].y - o[2].x); w[2] = t; }          // h(1 - i)
    { V t; t.x = s1 * o[3].x + c1 * o[3].y; t.y = s1 * o[3].y - c1 * o[3].x; w[3] = t; }   // (s1 - i c1)
    w[4] = mul_mi(o[4]);                                                                  // -i
    { V t; t.x = -s1 * o[5].x + c1 * o[5].y; t.y = -s1 * o[5].y - c1 * o[5].x; w[5] = t; } // (-s1 - i c1)
    { V t; t.x = h * (o[6].y - o[6].x); t.y = -h * (o[6].x + o[6].y); w[6] = t; }         // h(-1 - i)
    { V t; t.x = -c1 * o[7].x + s1 * o[7].y; t.y = -c1 * o[7].y - s1 * o[7].x; w[7] = t; } // (-c1 - i s1)
#pragma unroll
    for (int k = 0; k < 8; ++k) { v[k] = cadd(e[k], w[k]); v[k + 8] = csub(e[k], w[k]); }
}

// y_k = E_k + W_32^k O_k, y_{k+16} = E_k - W_32^k O_k with E, O the 16-point
// DFTs of the even and odd samples; W_32^k = cos(k pi/16) - i sin(k pi/16).
template <typename V> __device__ __forceinline__ void dft32(V* v) {
    using S = decltype(v[0].x);
    // cos(k pi/16) and sin(k pi/16) for k = 0..8
    const S C[9] = {S(1), S(0.980785280403230449126182236134239037), S(0.923879532511286756128183189396788287),
                    S(0.831469612302545237078788377617905757), S(0.707106781186547524400844362104849039),
                    S(0.555570233019602224742830813948532874), S(0.382683432365089771728459984030398867),
                    S(0.195090322016128267848284868477022241), S(0)};
    const S Sn[9] = {S(0), S(0.195090322016128267848284868477022241), S(0.382683432365089771728459984030398867),
                     S(0.555570233019602224742830813948532874), S(0.707106781186547524400844362104849039),
                     S(0.831469612302545237078788377617905757), S(0.923879532511286756128183189396788287),
                     S(0.980785280403230449126182236134239037), S(1)};
    V e[16], o[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) { e[k] = v[2 * k]; o[k] = v[2 * k + 1]; }
    dft16(e);
    dft16(o);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        V w;
        if (k == 0) {
            w = o[0];
        } else if (k == 8) {
            w = mul_mi(o[8]);
        } else {
            // cos(k pi/16) = -cos((16-k) pi/16), sin(k pi/16) = sin((16-k) pi/16) for k > 8
            const S c = k < 8 ? C[k] : -C[16 - k];
            const S sn = k < 8 ? Sn[k] : Sn[16 - k];
            w.x = c * o[k].x + sn * o[k].y;
            w.y = c * o[k].y - sn * o[k].x;
        }
        v[k] = cadd(e[k], w);
        v[k + 16] = csub(e[k], w);
    }
}

template <int R, typename V> __device__ __forceinline__ void dft(V* v) {
    if constexpr (R == 2) dft2(v[0], v[1]);
    else if constexpr (R == 3) dft3(v);
    else if constexpr (R == 4) dft4(v);
    else if constexpr (R == 5) dft5(v);
    else if constexpr (R == 8) dft8(v);
    else if constexpr (R == 16) dft16(v);
    else if constexpr (R == 32) dft32(v);
    else static_assert(R == 2, "unsupported radix");
}

// ---- LDS layout of a tile ----------------------------------------------------
// Element j of a line sits at lds_idx(j): one pad slot per 16 elements keeps
// the stride-R scatter of the early Stockham stages off a single bank.  The
// line pitch is odd so the W lines of a column tile fall on different banks.
__host__ __device__ constexpr int lds_idx(int j) { return j + (j >> 4); }
__host__ __device__ constexpr int Pitch_value(int L) { return (lds_idx(L - 1) + 1) | 1; }
// LDS of a tile of W lines: the lines, then the twiddle table W_L^m (m < L),
// copied in at the start of the tile so the radix stages read twiddles from
// LDS instead of waiting on global memory after each barrier.  A tile whose
// exchanges run in P parts holds only L/P positions of each line.
__host__ __device__ constexpr int line_pitch(int L, int P) { return Pitch_value(L / P); }
__host__ __device__ constexpr int64_t tile_lds_elems(int W, int L, int P = 1) {
    return (int64_t)W * line_pitch(L, P) + L;
}
// A transposing pass adds a table of one 64-bit row offset per line (W
// elements of at least 8 bytes).
__host__ __device__ constexpr int64_t tile_lds_elems_transpose(int W, int L, int P = 1) {
    return tile_lds_elems(W, L, P) + W;
}

// ---- Stockham stages ---------------------------------------------------------
// A thread of rank t (0 <= t < TPL) within its line owns butterflies
// b = t + i*TPL of every stage.  The first stage reads its inputs from `src`
// (HBM or LDS), the last stage hands its outputs to `sink`; between stages
// the values pass through the LDS copy `line` of the thread's line, and the
// stage functions hand their register arrays on explicitly.
template <typename V, int L, int TPL, int R>
struct StageShape {
    static constexpr int B = L / R;                 // butterflies in the stage
    static constexpr int NB = (B + TPL - 1) / TPL;  // butterflies per thread
    static constexpr bool EXACT = (B % TPL) == 0;
};

template <int R, int... Rest> struct FirstRadix { static constexpr int value = R; };

// The register array of one thread in a stage of radix R: R values for each
// of its butterflies.
template <typename V, int L, int TPL, int R>
using StageRegs = V[StageShape<V, L, TPL, R>::NB][R];

// LDS exchange between a stage with span NS and radix R (outputs v) and the
// next stage of radix R2 (inputs u).  The outputs go to their Stockham
// positions (b div NS)*NS*R + (b mod NS) + r*NS; the next stage reads
// b2 + r2*L/R2.
//
// Parts: the exchange may run in P phases over the positions [p*L/P,
// (p+1)*L/P) of every line, so LDS holds only L/P positions per line.  The
// output block of butterfly b, NS*R consecutive positions, lies in part
// b div (L/(R*P)) when NS*R divides L/P, and the next stage's element r2
// lies in part r2 div (R2/P) when P divides R2.  Phase p writes the
// butterflies of part p and reads elements r2 of part p; every thread takes
// part in every phase, so each exchange is 2*P barriers for all threads.
template <typename V, int L, int TPL, int NS, int R, int R2, int P>
__device__ __forceinline__ void exchange_parts(V* __restrict__ line, int t, bool act,
                                               const StageRegs<V, L, TPL, R>& v, StageRegs<V, L, TPL, R2>& u) {
    using S1 = StageShape<V, L, TPL, R>;
    using S2 = StageShape<V, L, TPL, R2>;
    constexpr int PART = L / P;      // positions per part
    constexpr int BP = S1::B / P;    // writing butterflies per part
    constexpr int RP = R2 / P;       // reading elements per part
    // b = t + i*TPL with t < TPL: when TPL divides BP the part of butterfly b
    // is (i*TPL) div BP, known per register slot at compile time, so each
    // slot's outputs are dead after its own phase
    constexpr bool BY_SLOT = BP % TPL == 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int i = 0; i < S1::NB; ++i) {
            const int b = t + i * TPL;
            const bool in_part = P == 1 || (BY_SLOT ? (i * TPL) / BP == p : b / BP == p);
            if (act && (S1::EXACT || b < S1::B) && in_part) {
                const int base = (b / NS) * NS * R + (b % NS) - p * PART;
#pragma unroll
                for (int r = 0; r < R; ++r) line[lds_idx(base + r * NS)] = v[i][r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < S2::NB; ++i) {
            const int b = t + i * TPL;
            if (act && (S2::EXACT || b < S2::B)) {
#pragma unroll
                for (int r = p * RP; r < (p + 1) * RP; ++r) u[i][r] = line[lds_idx(b + r * S2::B - p * PART)];
            }
        }
        __syncthreads();
    }
}

// Whether an exchange after a stage of span NS and radix R, before a stage
// of radix R2, can run in P parts (the host checks the same for a kernel).
template <int L, int NS, int R, int R2, int P>
__host__ __device__ constexpr bool exchange_splits() {
    return P == 1 || (L % P == 0 && R2 % P == 0 && (L / P) % (NS * R) == 0);
}

template <typename V, int L, int TPL, int P, int NS, int R, int R2>
__device__ __forceinline__ void exchange(V* __restrict__ line, int t, bool act, const StageRegs<V, L, TPL, R>& v,
                                         StageRegs<V, L, TPL, R2>& u) {
    static_assert(exchange_splits<L, NS, R, R2, P>(), "exchange cannot run in P parts");
    exchange_parts<V, L, TPL, NS, R, R2, P>(line, t, act, v, u);
}

// Sinks that take the outputs in parts: a sink type with a static kParts > 1
// receives the outputs of part p (indices [p*L/kParts, (p+1)*L/kParts)) and
// then its flush(p), between barriers, part after part (a line's outputs
// then need only L/kParts slots of LDS at a time).  Other sinks take every
// output at once.
template <typename S, typename = void> struct SinkParts { static constexpr int value = 1; };
template <typename S> struct SinkParts<S, decltype((void)S::kParts)> { static constexpr int value = S::kParts; };

// The last stage's outputs j = b + r*L/R to the sink.  Output j lies in part
// r div (R/kParts) when kParts divides R.
template <typename V, int L, int TPL, int R, typename Sink>
__device__ __forceinline__ void emit_outputs(StageRegs<V, L, TPL, R>& v, int t, bool act, Sink& sink) {
    using SH = StageShape<V, L, TPL, R>;
    constexpr int OP = SinkParts<Sink>::value;
    static_assert(R % OP == 0, "the last radix must split into the sink's parts");
#pragma unroll
    for (int p = 0; p < OP; ++p) {
#pragma unroll
        for (int i = 0; i < SH::NB; ++i) {
            const int b = t + i * TPL;
            if (act && (SH::EXACT || b < SH::B)) {
#pragma unroll
                for (int r = p * (R / OP); r < (p + 1) * (R / OP); ++r) sink(b + r * SH::B, v[i][r]);
            }
        }
        if constexpr (OP > 1) {
            __syncthreads();
            sink.flush(p);
            __syncthreads();
        }
    }
}

// Stage with span NS > 1 and radix R on the register inputs v: twiddles
// W_{Ns R}^(r (b mod Ns)) from the table W_L^m, the R-point DFT, then either
// the sink (last stage: natural-order index j = b + r*L/R) or the exchange
// into the next stage.
template <typename V, int L, int TPL, int P, int NS, int R, int... Rest, typename Sink>
__device__ __forceinline__ void stage_regs(StageRegs<V, L, TPL, R>& v, V* __restrict__ line,
                                           const V* __restrict__ tw, int t, bool act, Sink& sink) {
    using SH = StageShape<V, L, TPL, R>;
    constexpr int STEP = L / (NS * R);   // W_{Ns R}^e = W_L^(e STEP)
#pragma unroll
    for (int i = 0; i < SH::NB; ++i) {
        const int b = t + i * TPL;
        if (act && (SH::EXACT || b < SH::B)) {
            const int k = b % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw[r * k * STEP]);
            dft<R>(v[i]);
        }
    }
    if constexpr (sizeof...(Rest) == 0) {
        static_assert(NS * R == L, "last stage must complete the transform");
        emit_outputs<V, L, TPL, R>(v, t, act, sink);
    } else {
        constexpr int R2 = FirstRadix<Rest...>::value;
        StageRegs<V, L, TPL, R2> u;
        exchange<V, L, TPL, P, NS, R, R2>(line, t, act, v, u);
        stage_regs<V, L, TPL, P, NS * R, Rest...>(u, line, tw, t, act, sink);
    }
}

// First-stage inputs of the thread's butterflies: v[i][r] = src(b + r*L/R).
template <typename V, int L, int TPL, int R, typename Src>
__device__ __forceinline__ void load_first(StageRegs<V, L, TPL, R>& v, int t, bool act, Src& src) {
    using SH = StageShape<V, L, TPL, R>;
#pragma unroll
    for (int i = 0; i < SH::NB; ++i) {
        const int b = t + i * TPL;
        if (act && (SH::EXACT || b < SH::B)) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = src(b + r * SH::B);
        }
    }
}

// The 1-D FFT of the thread's line from its first-stage inputs v (already
// loaded).  IN_LDS: the inputs came from LDS (so the first exchange's writes
// wait for every read); OUT_LDS: `sink` writes LDS (the last exchange ends
// with a barrier, so every LDS read precedes it).  Lanes with act == false
// only take part in the barriers.
template <typename V, int L, int TPL, int P, bool IN_LDS, bool OUT_LDS, int R, int... Rest, typename Sink>
__device__ __forceinline__ void fft_from_regs(StageRegs<V, L, TPL, R>& v, V* __restrict__ line,
                                              const V* __restrict__ tw, int t, bool act, Sink& sink) {
    using SH = StageShape<V, L, TPL, R>;
#pragma unroll
    for (int i = 0; i < SH::NB; ++i) {
        const int b = t + i * TPL;
        if (act && (SH::EXACT || b < SH::B)) dft<R>(v[i]);   // span 1: no twiddles
    }
    if constexpr (sizeof...(Rest) == 0) {
        // a single stage: output j = r (one butterfly, b = 0)
        if constexpr (OUT_LDS || IN_LDS) __syncthreads();
        emit_outputs<V, L, TPL, R>(v, t, act, sink);
    } else {
        if constexpr (IN_LDS) __syncthreads();
        constexpr int R2 = FirstRadix<Rest...>::value;
        StageRegs<V, L, TPL, R2> u;
        exchange<V, L, TPL, P, 1, R, R2>(line, t, act, v, u);
        stage_regs<V, L, TPL, P, R, Rest...>(u, line, tw, t, act, sink);
    }
}

// Whole 1-D FFT of the thread's line: first-stage loads from `src`, then
// fft_from_regs.  P: the parts every LDS exchange runs in.
template <typename V, int L, int TPL, int P, bool IN_LDS, bool OUT_LDS, int R, int... Rest, typename Src,
          typename Sink>
__device__ __forceinline__ void run_fft(V* __restrict__ line, const V* __restrict__ tw, int t, bool act, Src& src,
                                        Sink& sink) {
    StageRegs<V, L, TPL, R> v;
    load_first<V, L, TPL, R>(v, t, act, src);
    fft_from_regs<V, L, TPL, P, IN_LDS, OUT_LDS, R, Rest...>(v, line, tw, t, act, sink);
}

template <int... Rs> struct RadixProduct;
template <> struct RadixProduct<> { static constexpr int value = 1; };
template <int R, int... Rest> struct RadixProduct<R, Rest...> {
    static constexpr int value = R * RadixProduct<Rest...>::value;
};

// ---- pass arguments --------------------------------------------------------
struct PassArgs {
    const void* in;
    void* out;
    const void* tw;     // W_L^m, m < L, in the pass precision
    int64_t nlines;     // M1 * M2 (M1 * lpm for a column block)
    int64_t M2;         // element stride of the axis (1: contiguous lines)
    // strided lines (mode 1): lines per m1, and a column block: with
    // blk_logw >= 0, line v of an m1 lies at
    // m2 = (v >> blk_logw) * blk_ld + blk_off + (v & (2^blk_logw - 1)),
    // the lines of 2^blk_logw consecutive columns out of every blk_ld
    // (without a block, lpm == M2 and m2 = v)
    int64_t lpm;
    int64_t blk_ld, blk_off;
    int blk_logw;
    int64_t X, Y;       // transposing passes: line m1*M2 + m2 is the contiguous row
                        // m1*M2 + (m2 mod X)*Y + m2 div X of the other buffer
    int logW;           // log2 of lines per workgroup
    int mode;           // 0: contiguous lines (M2 == 1), 1: strided lines,
                        // 2: rows in, strided lines out, 3: strided lines in, rows out
    int xcd_remap;      // 1: tiles in contiguous runs per XCD (xcd_tile)
    int stream_io;      // 1: grid data loaded and stored with streaming (non-temporal) accesses
    int conj_in;        // negate imaginary parts on load
    int conj_out;       // negate imaginary parts on store
    double scale;       // multiply on store
};

// Workgroups go to the 8 XCDs round-robin in launch order.  With remap, the
// first 8*floor(n/8) of n workgroups take tiles so that each XCD works through
// one contiguous run of tiles (workgroup i: tile (i mod 8)*floor(n/8) +
// i div 8), the rest keep their own index; a bijection on [0, n).
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t i, int64_t n, int remap) {
    if (!remap) return i;
    const int64_t q = n / kXcds;
    return i < kXcds * q ? (i % kXcds) * q + i / kXcds : i;
}

template <typename V> __device__ __forceinline__ V fix_in(V x, int conj) {
    if (conj) x.y = -x.y;
    return x;
}
template <typename V, typename S> __device__ __forceinline__ V fix_out(V x, int conj, S scale) {
    if (conj) x.y = -x.y;
    x.x *= scale;
    x.y *= scale;
    return x;
}

// Grid data is read once and written once per pass.  A pass can access it
// with non-temporal (streaming) loads and stores (PassArgs::stream_io): the
// lines are then not kept in the caches for reuse.  On MI355X that raises the
// rate of the strided tile loads and stores of grids much larger than the
// 256 MB Infinity Cache, and lowers it for grids that fit there, whose next
// pass reads what the previous one left in the cache.
template <typename S> struct StreamVec { typedef S type __attribute__((vector_size(2 * sizeof(S)))); };
template <typename V> __device__ __forceinline__ V load_stream(const V* p) {
    using S = decltype(V{}.x);
    using E = typename StreamVec<S>::type;
    const E e = __builtin_nontemporal_load(reinterpret_cast<const E*>(p));
    V v;
    v.x = e[0];
    v.y = e[1];
    return v;
}
template <typename V> __device__ __forceinline__ void store_stream(V* p, V v) {
    using S = decltype(V{}.x);
    using E = typename StreamVec<S>::type;
    E e;
    e[0] = v.x;
    e[1] = v.y;
    __builtin_nontemporal_store(e, reinterpret_cast<E*>(p));
}
// Load / store of grid data: streaming when nt (uniform across the workgroup).
template <typename V> __device__ __forceinline__ V load_io(const V* p, bool nt) {
    return nt ? load_stream(p) : *p;
}
template <typename V> __device__ __forceinline__ void store_io(V* p, V v, bool nt) {
    if (nt) store_stream(p, v);
    else *p = v;
}

// Store of one element to HBM.  COHERENT stores are agent-scope relaxed
// atomics: they write through the XCD's L2, so data another workgroup will
// read after a release/acquire handshake never sits dirty in one L2 and the
// release has nothing to write back.
template <bool COHERENT, typename V> __device__ __forceinline__ void store_elem(V* p, V x);
template <> __device__ __forceinline__ void store_elem<false, float2>(float2* p, float2 x) { *p = x; }
template <> __device__ __forceinline__ void store_elem<false, double2>(double2* p, double2 x) { *p = x; }
template <> __device__ __forceinline__ void store_elem<true, float2>(float2* p, float2 x) {
    uint64_t bits;
    __builtin_memcpy(&bits, &x, sizeof bits);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <> __device__ __forceinline__ void store_elem<true, double2>(double2* p, double2 x) {
    uint64_t bx, by;
    __builtin_memcpy(&bx, &x.x, sizeof bx);
    __builtin_memcpy(&by, &x.y, sizeof by);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), bx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p) + 1, by, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Load and store of grid data in a pass tile: streaming when the pass asks
// for it, never in the batch executors' coherent form (whose tiles read what
// other workgroups of the same launch wrote, after the acquire that orders it).
template <bool COHERENT, typename V> __device__ __forceinline__ V load_elem(const V* p, bool nt) {
    if constexpr (COHERENT) return *p;
    else return load_io(p, nt);
}
template <bool COHERENT, typename V> __device__ __forceinline__ void store_elem_io(V* p, V x, bool nt) {
    if constexpr (COHERENT) store_elem<true>(p, x);
    else store_io(p, x, nt);
}

// Contiguous lines with fewer than this many threads per line are staged
// through LDS with a flat coalesced copy (direct loads would touch one
// element per line per lane).
constexpr int kDirectRowMinTpl = 16;

// The thread's index in one tile's code.  In a loop that runs tile after
// tile over every kernel case (the level-synchronous batch executor) it is
// made opaque with an empty asm, so that each case's per-thread index math
// stays inside its tile instead of being hoisted out of the loop for all the
// cases at once, where it would stay live across the loop and spill.
#ifndef OFFT_OPAQUE_VGPR   // the CPU emulation of this header defines it away
#define OFFT_OPAQUE_VGPR(x) asm volatile("" : "+v"(x))
#endif
template <bool OPAQUE>
__device__ __forceinline__ int tile_thread_index() {
    int tid = (int)threadIdx.x;
    if constexpr (OPAQUE) OFFT_OPAQUE_VGPR(tid);
    return tid;
}

// Device body of one axis pass for one tile of W = 2^logW lines starting at
// line l0.  Threads: W * TPL.  lds: tile_lds_elems(W, L) elements.
//   strided lines:     lanes walk the W lines (consecutive columns of a row),
//                      first/last stage straight from/to HBM.
//   contiguous lines:  lanes walk along the line; first/last stage straight
//                      from/to HBM when TPL >= kDirectRowMinTpl, else the tile
//                      is staged through LDS as one contiguous block.
// Threads beyond W*TPL (possible when a larger workgroup runs this tile, as in
// the persistent batch executor) only take part in the barriers.
template <typename V, bool COHERENT, bool LOOPED, int L, int TPL, int P, int... Rs>
__device__ __forceinline__ void pass_tile_impl(const PassArgs& a, V* __restrict__ lds, int64_t l0) {
    using S = decltype(V{}.x);
    static_assert(RadixProduct<Rs...>::value == L, "radix sequence must multiply to L");
    constexpr int LP = line_pitch(L, P);
    const int W = 1 << a.logW;
    const int tid = tile_thread_index<LOOPED>();
    const int64_t rem = a.nlines - l0;
    const int nl = rem < W ? (int)rem : W;
    const V* __restrict__ in = static_cast<const V*>(a.in);
    V* __restrict__ out = static_cast<V*>(a.out);
    const V* tw = static_cast<const V*>(a.tw);
    const int cin = a.conj_in, cout = a.conj_out;
    const S scale = (S)a.scale;
    const bool active = tid < W * TPL;
    const bool nt = !COHERENT && a.stream_io;
    if constexpr (sizeof...(Rs) > 1) {
        // stage the twiddle table; the first barrier inside run_fft (after the
        // first stage, which needs no twiddles) orders it before any use
        V* twl = lds + W * LP;
        for (int i = tid; i < L; i += (int)blockDim.x) twl[i] = tw[i];
        tw = twl;
    }

    if (a.mode == 1) {
        const int w = tid & (W - 1);
        const int t = tid >> a.logW;
        const bool ok = active && w < nl;
        const int64_t l = l0 + (ok ? w : 0);   // rows beyond the tail read line l0, store nothing
        const int64_t m1 = l / a.lpm, v = l - m1 * a.lpm;
        const int64_t m2 = a.blk_logw < 0 ? v
                                          : (v >> a.blk_logw) * a.blk_ld + a.blk_off +
                                                (v & ((int64_t(1) << a.blk_logw) - 1));
        const int64_t base = m1 * (int64_t)L * a.M2 + m2;
        const int64_t M2 = a.M2;
        const V* g = in + base;
        V* go = out + base;
        auto src = [&](int j) { return fix_in(load_elem<COHERENT>(g + (int64_t)j * M2, nt), cin); };
        auto sink = [&](int j, V x) {
            if (ok) store_elem_io<COHERENT>(go + (int64_t)j * M2, fix_out(x, cout, scale), nt);
        };
        run_fft<V, L, TPL, P, false, false, Rs...>(lds + w * LP, tw, t, active, src, sink);
        return;
    }
    // contiguous lines keep whole lines in LDS: kernels with parts serve strided lines only
    if constexpr (P == 1) {
        const int t = tid % TPL, w = active ? tid / TPL : 0;
        V* line = lds + w * LP;
        if constexpr (TPL >= kDirectRowMinTpl) {
            const bool ok = active && tid / TPL < nl;
            const V* g = in + (l0 + (ok ? w : 0)) * L;
            V* go = out + (l0 + w) * L;
            auto src = [&](int j) { return fix_in(load_elem<COHERENT>(g + j, nt), cin); };
            auto sink = [&](int j, V x) {
                if (ok) store_elem_io<COHERENT>(go + j, fix_out(x, cout, scale), nt);
            };
            run_fft<V, L, TPL, 1, false, false, Rs...>(line, tw, t, active, src, sink);
        } else {
            // stage the contiguous block of nl*L elements through LDS
            const int NT = W * TPL;
            const V* g = in + l0 * L;
            V* go = out + l0 * L;
            if (active) {
                for (int f = tid; f < nl * L; f += NT) {
                    const int lw = f / L, j = f - lw * L;
                    lds[lw * LP + lds_idx(j)] = fix_in(load_elem<COHERENT>(g + f, nt), cin);
                }
            }
            __syncthreads();
            auto src = [&](int j) { return line[lds_idx(j)]; };
            auto sink = [&](int j, V x) { line[lds_idx(j)] = x; };
            run_fft<V, L, TPL, 1, true, true, Rs...>(line, tw, t, active, src, sink);
            __syncthreads();
            if (active) {
                for (int f = tid; f < nl * L; f += NT) {
                    const int lw = f / L, j = f - lw * L;
                    store_elem_io<COHERENT>(go + f, fix_out(lds[lw * LP + lds_idx(j)], cout, scale), nt);
                }
            }
        }
    }
}

// Row-side stores of a transposing pass whose last stage emits in P parts:
// part p of every line goes to its line's LDS slots, then the W half (or
// quarter) rows leave with a flat coalesced copy.
template <typename V, int L, int P>
struct RowPartSink {
    static constexpr int kParts = P;
    static constexpr int PART = L / P;
    static constexpr int LP = line_pitch(L, P);
    V* line;                         // this thread's line slots
    V* lds;                          // the tile (line w at lds + w*LP)
    V* out;
    const int64_t* rows;             // element offset of each line's row
    int nl, tid, nt, cout;
    decltype(V{}.x) scale;
    bool active;
    bool stream;                     // streaming stores
    __device__ __forceinline__ void operator()(int j, V x) {
        line[lds_idx(j % PART)] = fix_out(x, cout, scale);
    }
    __device__ __forceinline__ void flush(int p) {
        if (!active) return;
        for (int f = tid; f < nl * PART; f += nt) {
            const int lw = f / PART, jj = f - lw * PART;
            store_io(out + rows[lw] + p * PART + jj, lds[lw * LP + lds_idx(jj)], stream);
        }
    }
};

// One tile of a transposing pass (modes 2 and 3): W lines whose strided side
// follows the [M1][L][M2] view (line l = m1*M2 + m2 at m1*L*M2 + m2, stride
// M2) while the other buffer holds each line as the contiguous row
// m1*M2 + (m2 mod X)*Y + m2 div X.  Mode 2 reads the rows and writes the
// strided lines, mode 3 the reverse.  The row side goes through LDS with a
// flat coalesced copy (consecutive lanes on consecutive elements of a row);
// the strided side goes straight between registers and HBM with lanes walking
// the W columns, as in a strided pass.  With P > 1 the exchanges run in P
// parts and the row side moves part by part (the first radix and the last
// radix must split into P), so the tile needs LDS for only L/P elements of
// each line.  Threads: W * TPL; lds: tile_lds_elems_transpose(W, L, P)
// elements.  Never in place.
template <typename V, int L, int TPL, int P, int... Rs>
__device__ __forceinline__ void pass_tile_transpose(const PassArgs& a, V* __restrict__ lds, int64_t l0) {
    using S = decltype(V{}.x);
    static_assert(RadixProduct<Rs...>::value == L, "radix sequence must multiply to L");
    constexpr int LP = line_pitch(L, P);
    constexpr int PART = L / P;
    const int W = 1 << a.logW;
    const int NT = W * TPL;
    const int tid = threadIdx.x;
    const int64_t rem = a.nlines - l0;
    const int nl = rem < W ? (int)rem : W;
    const V* __restrict__ in = static_cast<const V*>(a.in);
    V* __restrict__ out = static_cast<V*>(a.out);
    const V* tw = static_cast<const V*>(a.tw);
    const int cin = a.conj_in, cout = a.conj_out;
    const S scale = (S)a.scale;
    const bool active = tid < NT;
    const bool nts = a.stream_io != 0;
    const int64_t M2 = a.M2;
    if constexpr (sizeof...(Rs) > 1) {
        V* twl = lds + W * LP;
        for (int i = tid; i < L; i += (int)blockDim.x) twl[i] = tw[i];
        tw = twl;
    }
    // element offset of each line's row in the row-side buffer
    int64_t* rows = reinterpret_cast<int64_t*>(lds + W * LP + L);
    if (tid < nl) {
        const int64_t l = l0 + tid;
        const int64_t m1 = l / M2, m2 = l - m1 * M2;
        rows[tid] = (m1 * M2 + (m2 % a.X) * a.Y + m2 / a.X) * (int64_t)L;
    }
    __syncthreads();
    const int w = tid & (W - 1);
    const int t = tid >> a.logW;
    const bool ok = active && w < nl;
    const int64_t l = l0 + (ok ? w : 0);   // rows beyond the tail compute on line l0, store nothing
    const int64_t m1 = l / M2, m2 = l - m1 * M2;
    const int64_t base = m1 * (int64_t)L * M2 + m2;
    V* line = lds + w * LP;
    if (a.mode == 2) {
        V* go = out + base;
        auto sink = [&](int j, V x) {
            if (ok) store_io(go + (int64_t)j * M2, fix_out(x, cout, scale), nts);
        };
        if constexpr (P == 1) {
            if (active) {
                for (int f = tid; f < nl * L; f += NT) {
                    const int lw = f / L, j = f - lw * L;
                    lds[lw * LP + lds_idx(j)] = fix_in(load_io(in + rows[lw] + j, nts), cin);
                }
            }
            __syncthreads();
            auto src = [&](int j) { return line[lds_idx(j)]; };
            run_fft<V, L, TPL, 1, true, false, Rs...>(line, tw, t, active, src, sink);
        } else {
            // the first stage's inputs part by part: input j = b + r*L/R0
            // lies in part r div (R0/P)
            constexpr int R0 = FirstRadix<Rs...>::value;
            static_assert(R0 % P == 0, "the first radix must split into the parts");
            using SH = StageShape<V, L, TPL, R0>;
            StageRegs<V, L, TPL, R0> v;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (active) {
                    for (int f = tid; f < nl * PART; f += NT) {
                        const int lw = f / PART, jj = f - lw * PART;
                        lds[lw * LP + lds_idx(jj)] = fix_in(load_io(in + rows[lw] + p * PART + jj, nts), cin);
                    }
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < SH::NB; ++i) {
                    const int b = t + i * TPL;
                    if (active && (SH::EXACT || b < SH::B)) {
#pragma unroll
                        for (int r = p * (R0 / P); r < (p + 1) * (R0 / P); ++r)
                            v[i][r] = line[lds_idx(b + r * SH::B - p * PART)];
                    }
                }
                __syncthreads();
            }
            fft_from_regs<V, L, TPL, P, false, false, Rs...>(v, line, tw, t, active, sink);
        }
    } else {
        const V* g = in + base;
        auto src = [&](int j) { return fix_in(load_io(g + (int64_t)j * M2, nts), cin); };
        if constexpr (P == 1) {
            auto sink = [&](int j, V x) { line[lds_idx(j)] = fix_out(x, cout, scale); };
            run_fft<V, L, TPL, 1, false, true, Rs...>(line, tw, t, active, src, sink);
            __syncthreads();
            if (active) {
                for (int f = tid; f < nl * L; f += NT) {
                    const int lw = f / L, j = f - lw * L;
                    store_io(out + rows[lw] + j, lds[lw * LP + lds_idx(j)], nts);
                }
            }
        } else {
            RowPartSink<V, L, P> sink{line, lds, out, rows, nl, tid, NT, cout, scale, active, nts};
            run_fft<V, L, TPL, P, false, true, Rs...>(line, tw, t, active, src, sink);
        }
    }
}

// One tile of an axis pass with ordinary stores (stand-alone pass kernels).
template <typename V, int L, int TPL, int... Rs>
__device__ __forceinline__ void pass_tile(const PassArgs& a, V* __restrict__ lds, int64_t l0) {
    pass_tile_impl<V, false, false, L, TPL, 1, Rs...>(a, lds, l0);
}

// One tile of a strided pass whose LDS exchanges run in P parts (stand-alone
// pass kernels of lengths whose radix sequence allows it).
template <typename V, int L, int TPL, int P, int... Rs>
__device__ __forceinline__ void pass_tile_parts(const PassArgs& a, V* __restrict__ lds, int64_t l0) {
    pass_tile_impl<V, false, false, L, TPL, P, Rs...>(a, lds, l0);
}

// One tile with write-through stores (batch executors, whose tiles are read
// by other workgroups of the same launch).
template <typename V, int L, int TPL, int... Rs>
__device__ __forceinline__ void pass_tile_coherent(const PassArgs& a, V* __restrict__ lds, int64_t l0) {
    pass_tile_impl<V, true, false, L, TPL, 1, Rs...>(a, lds, l0);
}

// One tile with ordinary stores inside a loop over tiles of every kernel
// case (the level-synchronous batch executor).
template <typename V, int L, int TPL, int... Rs>
__device__ __forceinline__ void pass_tile_looped(const PassArgs& a, V* __restrict__ lds, int64_t l0) {
    pass_tile_impl<V, false, true, L, TPL, 1, Rs...>(a, lds, l0);
}

}  // namespace offt
