/*
 * offt_oracle.c -- plain, slow, fp64 CPU oracle for the 3-D complex-to-complex
 * DFT.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU
 * baseline leg of the benchmark call it; the GPU library never does, and the
 * two share no source.
 *
 * What is computed (Duy & Ozaki, "Performance Tuning of a Parallel 3-D FFT
 * Package OpenFFT", Sec. 2 and Sec. 3.1.1):
 *   - a grid A(a,b,c) of Na x Nb x Nc complex values stored row-major with c
 *     fastest: offset a*Nb*Nc + b*Nc + c (Sec. 2, Eq. 1);
 *   - its 3-D DFT, obtained in the paper by 1-D transforms "in a particular
 *     dimension" followed by a transpose while dimensions remain (Sec. 3.1.1,
 *     calculation flow), in the transpose order abc -> cab -> cba (Sec. 2), i.e.
 *     the c axis first, then b, then a.  Separability of the DFT makes that
 *     composition equal to the plain definition
 *       X[ka,kb,kc] = sum_a sum_b sum_c x[a,b,c] W_Na^(a ka) W_Nb^(b kb) W_Nc^(c kc),
 *     W_n = exp(sign * 2 pi i / n), sign = -1 forward, +1 backward (FFTW's
 *     convention; the paper uses FFTW as its 1-D engine and states no sign).
 *
 * Data: interleaved (re, im) binary64, i.e. double[2*N].
 *
 * Parts:
 *   oracle_root_table   W_n^m for m < n, exact at the quarter points
 *   oracle_dft3_brute   (O1) the triple sum itself, O(N^2)
 *   oracle_dft3_axes    (O2) naive O(n^2) DFT along c, then b, then a
 *   oracle_fft3         (O3) recursive smallest-prime-first mixed-radix FFT
 *                       (radix 2/3/5) along c, then b, then a
 *   oracle_dft3_line    X[ka,kb,0..Nc) from the definition, O(N + Nc^2)
 *   oracle_dft3_point   one X[ka,kb,kc] from the definition, O(N)
 *
 * Every function returns 0 on success, -1 on a bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cpx;

static inline cpx cmul(cpx a, cpx b) {
    cpx r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}
static inline cpx cadd(cpx a, cpx b) { cpx r = { a.re + b.re, a.im + b.im }; return r; }

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* T[m] = exp(sign*2*pi*i*m/n), m < n.  The values at m = 0, n/4, n/2, 3n/4
 * (where those are integers) are set exactly to 1, -+i, -1, +-i. */
static int root_table(int64_t n, int sign, cpx* T) {
    if (n < 1 || (sign != 1 && sign != -1)) return -1;
    const double twopi = 6.283185307179586476925286766559;
    for (int64_t m = 0; m < n; ++m) {
        double ang = twopi * (double)m / (double)n;
        T[m].re = cos(ang);
        T[m].im = sign * sin(ang);
    }
    T[0].re = 1.0; T[0].im = 0.0;
    if (n % 2 == 0) { T[n / 2].re = -1.0; T[n / 2].im = 0.0; }
    if (n % 4 == 0) {
        T[n / 4].re = 0.0;      T[n / 4].im = (double)sign;
        T[3 * n / 4].re = 0.0;  T[3 * n / 4].im = -(double)sign;
    }
    return 0;
}

int oracle_root_table(int64_t n, int sign, double* out) {
    return root_table(n, sign, (cpx*)out);
}

/* ---- O1: brute force ---------------------------------------------------- */
int oracle_dft3_brute(const double* xin, double* yout, int64_t Na, int64_t Nb,
                      int64_t Nc, int sign, int nthreads) {
    if (Na < 1 || Nb < 1 || Nc < 1 || (sign != 1 && sign != -1)) return -1;
    const cpx* x = (const cpx*)xin;
    cpx* y = (cpx*)yout;
    cpx* Ta = malloc(sizeof(cpx) * Na);
    cpx* Tb = malloc(sizeof(cpx) * Nb);
    cpx* Tc = malloc(sizeof(cpx) * Nc);
    if (!Ta || !Tb || !Tc) { free(Ta); free(Tb); free(Tc); return -1; }
    root_table(Na, sign, Ta);
    root_table(Nb, sign, Tb);
    root_table(Nc, sign, Tc);
    const int64_t N = Na * Nb * Nc;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < N; ++k) {
        const int64_t ka = k / (Nb * Nc), kb = (k / Nc) % Nb, kc = k % Nc;
        cpx acc = { 0.0, 0.0 };
        for (int64_t a = 0; a < Na; ++a)
            for (int64_t b = 0; b < Nb; ++b)
                for (int64_t c = 0; c < Nc; ++c) {
                    cpx w = cmul(cmul(Ta[(a * ka) % Na], Tb[(b * kb) % Nb]), Tc[(c * kc) % Nc]);
                    acc = cadd(acc, cmul(x[(a * Nb + b) * Nc + c], w));
                }
        y[k] = acc;
    }
    free(Ta); free(Tb); free(Tc);
    return 0;
}

/* ---- line helpers: gather/scatter one line of an axis ---------------------
 * axis 2 (c): stride 1, lines indexed by (a,b)
 * axis 1 (b): stride Nc, lines indexed by (a,c)
 * axis 0 (a): stride Nb*Nc, lines indexed by (b,c)                            */
static void line_geometry(int axis, int64_t Na, int64_t Nb, int64_t Nc, int64_t* n,
                          int64_t* nlines, int64_t* stride) {
    if (axis == 2) { *n = Nc; *nlines = Na * Nb; *stride = 1; }
    else if (axis == 1) { *n = Nb; *nlines = Na * Nc; *stride = Nc; }
    else { *n = Na; *nlines = Nb * Nc; *stride = Nb * Nc; }
}
static int64_t line_base(int axis, int64_t l, int64_t Nb, int64_t Nc) {
    if (axis == 2) return l * Nc;                       /* l = a*Nb + b */
    if (axis == 1) return (l / Nc) * Nb * Nc + l % Nc;  /* l = a*Nc + c */
    return l;                                           /* l = b*Nc + c */
}

/* ---- O2: naive per-axis DFT ----------------------------------------------- */
static void dft_naive(const cpx* x, cpx* y, int64_t n, const cpx* T) {
    for (int64_t k = 0; k < n; ++k) {
        cpx acc = { 0.0, 0.0 };
        for (int64_t j = 0; j < n; ++j) acc = cadd(acc, cmul(x[j], T[(j * k) % n]));
        y[k] = acc;
    }
}

/* ---- O3: recursive mixed-radix FFT ------------------------------------------
 * y[0..n) = DFT_n of the sequence x[0], x[s], x[2s], ...  Roots come from the
 * table T of the axis length nb: W_n^e = T[e * (nb / n)].
 * Decimation in time by the smallest prime factor p of n: the p subsequences
 * x_r[j] = x[(j p + r) s] are transformed recursively (length m = n/p) into
 * y[r m .. r m + m), then combined:
 *     out[k + q m] = sum_r W_n^(r (k + q m)) X_r[k],   k < m, q < p.
 * tmp holds at least n values; recursive calls finish before this level uses it. */
static int smallest_prime(int64_t n) {
    if (n % 2 == 0) return 2;
    if (n % 3 == 0) return 3;
    if (n % 5 == 0) return 5;
    return 0;
}
static void fft_rec(const cpx* x, int64_t s, cpx* y, int64_t n, const cpx* T, int64_t nb, cpx* tmp) {
    if (n == 1) { y[0] = x[0]; return; }
    const int p = smallest_prime(n);
    const int64_t m = n / p;
    for (int r = 0; r < p; ++r) fft_rec(x + r * s, s * p, y + r * m, m, T, nb, tmp);
    memcpy(tmp, y, sizeof(cpx) * n);
    const int64_t step = nb / n;
    for (int q = 0; q < p; ++q)
        for (int64_t k = 0; k < m; ++k) {
            cpx acc = { 0.0, 0.0 };
            for (int r = 0; r < p; ++r)
                acc = cadd(acc, cmul(T[((r * (k + q * m)) % n) * step], tmp[r * m + k]));
            y[k + q * m] = acc;
        }
}

static int check_smooth(int64_t n) {
    if (n < 1) return 0;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    while (n % 5 == 0) n /= 5;
    return n == 1;
}

/* Transform y in place along `axis` with method 0 = naive DFT, 1 = recursive FFT. */
static int axis_pass(cpx* y, int64_t Na, int64_t Nb, int64_t Nc, int axis, int sign, int method) {
    int64_t n, nlines, stride;
    line_geometry(axis, Na, Nb, Nc, &n, &nlines, &stride);
    if (n == 1) return 0;
    cpx* T = malloc(sizeof(cpx) * n);
    if (!T) return -1;
    root_table(n, sign, T);
    int fail = 0;
#pragma omp parallel
    {
        cpx* in = malloc(sizeof(cpx) * n);
        cpx* out = malloc(sizeof(cpx) * n);
        cpx* tmp = malloc(sizeof(cpx) * n);
        if (!in || !out || !tmp) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t l = 0; l < nlines; ++l) {
                const int64_t base = line_base(axis, l, Nb, Nc);
                for (int64_t j = 0; j < n; ++j) in[j] = y[base + j * stride];
                if (method == 0) dft_naive(in, out, n, T);
                else fft_rec(in, 1, out, n, T, n, tmp);
                for (int64_t j = 0; j < n; ++j) y[base + j * stride] = out[j];
            }
        }
        free(in); free(out); free(tmp);
    }
    free(T);
    return fail ? -1 : 0;
}

static int three_axes(const double* xin, double* yout, int64_t Na, int64_t Nb, int64_t Nc,
                      int sign, int nthreads, int method) {
    if (Na < 1 || Nb < 1 || Nc < 1 || (sign != 1 && sign != -1)) return -1;
    if (method == 1 && !(check_smooth(Na) && check_smooth(Nb) && check_smooth(Nc))) return -1;
    set_threads(nthreads);
    const int64_t N = Na * Nb * Nc;
    if (xin != yout) memcpy(yout, xin, sizeof(cpx) * N);
    cpx* y = (cpx*)yout;
    /* c first, then b, then a (transpose order abc -> cab -> cba). */
    if (axis_pass(y, Na, Nb, Nc, 2, sign, method)) return -1;
    if (axis_pass(y, Na, Nb, Nc, 1, sign, method)) return -1;
    if (axis_pass(y, Na, Nb, Nc, 0, sign, method)) return -1;
    return 0;
}

int oracle_dft3_axes(const double* x, double* y, int64_t Na, int64_t Nb, int64_t Nc,
                     int sign, int nthreads) {
    return three_axes(x, y, Na, Nb, Nc, sign, nthreads, 0);
}

int oracle_fft3(const double* x, double* y, int64_t Na, int64_t Nb, int64_t Nc,
                int sign, int nthreads) {
    return three_axes(x, y, Na, Nb, Nc, sign, nthreads, 1);
}

/* 1-D transform of `count` contiguous lines of length n (method as above). */
int oracle_fft1_lines(const double* x, double* y, int64_t n, int64_t count, int sign,
                      int nthreads, int method) {
    if (n < 1 || count < 0) return -1;
    if (method == 1 && !check_smooth(n)) return -1;
    set_threads(nthreads);
    if (x != y) memcpy(y, x, sizeof(cpx) * n * count);
    return axis_pass((cpx*)y, 1, count, n, 2, sign, method);
}

/* ---- sampled outputs from the definition -------------------------------------
 * u[c] = sum_a sum_b x[a,b,c] W_Na^(a ka) W_Nb^(b kb)   (all c at once)
 * X[ka,kb,kc] = sum_c u[c] W_Nc^(c kc)                                         */
int oracle_dft3_line(const double* xin, double* yline, int64_t Na, int64_t Nb, int64_t Nc,
                     int64_t ka, int64_t kb, int sign, int nthreads) {
    if (Na < 1 || Nb < 1 || Nc < 1 || (sign != 1 && sign != -1)) return -1;
    if (ka < 0 || ka >= Na || kb < 0 || kb >= Nb) return -1;
    const cpx* x = (const cpx*)xin;
    cpx* Ta = malloc(sizeof(cpx) * Na);
    cpx* Tb = malloc(sizeof(cpx) * Nb);
    cpx* Tc = malloc(sizeof(cpx) * Nc);
    cpx* u = calloc((size_t)Nc, sizeof(cpx));
    if (!Ta || !Tb || !Tc || !u) { free(Ta); free(Tb); free(Tc); free(u); return -1; }
    root_table(Na, sign, Ta);
    root_table(Nb, sign, Tb);
    root_table(Nc, sign, Tc);
    set_threads(nthreads);
#pragma omp parallel
    {
        cpx* up = calloc((size_t)Nc, sizeof(cpx));
#pragma omp for schedule(static)
        for (int64_t a = 0; a < Na; ++a)
            for (int64_t b = 0; b < Nb; ++b) {
                const cpx w = cmul(Ta[(a * ka) % Na], Tb[(b * kb) % Nb]);
                const cpx* row = x + (a * Nb + b) * Nc;
                for (int64_t c = 0; c < Nc; ++c) up[c] = cadd(up[c], cmul(row[c], w));
            }
#pragma omp critical
        for (int64_t c = 0; c < Nc; ++c) u[c] = cadd(u[c], up[c]);
        free(up);
    }
    cpx* y = (cpx*)yline;
    for (int64_t kc = 0; kc < Nc; ++kc) {
        cpx acc = { 0.0, 0.0 };
        for (int64_t c = 0; c < Nc; ++c) acc = cadd(acc, cmul(u[c], Tc[(c * kc) % Nc]));
        y[kc] = acc;
    }
    free(Ta); free(Tb); free(Tc); free(u);
    return 0;
}

int oracle_dft3_point(const double* xin, double* y1, int64_t Na, int64_t Nb, int64_t Nc,
                      int64_t ka, int64_t kb, int64_t kc, int sign) {
    if (Na < 1 || Nb < 1 || Nc < 1 || (sign != 1 && sign != -1)) return -1;
    if (ka < 0 || ka >= Na || kb < 0 || kb >= Nb || kc < 0 || kc >= Nc) return -1;
    const cpx* x = (const cpx*)xin;
    cpx* Ta = malloc(sizeof(cpx) * Na);
    cpx* Tb = malloc(sizeof(cpx) * Nb);
    cpx* Tc = malloc(sizeof(cpx) * Nc);
    if (!Ta || !Tb || !Tc) { free(Ta); free(Tb); free(Tc); return -1; }
    root_table(Na, sign, Ta);
    root_table(Nb, sign, Tb);
    root_table(Nc, sign, Tc);
    cpx acc = { 0.0, 0.0 };
    for (int64_t a = 0; a < Na; ++a)
        for (int64_t b = 0; b < Nb; ++b)
            for (int64_t c = 0; c < Nc; ++c) {
                cpx w = cmul(cmul(Ta[(a * ka) % Na], Tb[(b * kb) % Nb]), Tc[(c * kc) % Nc]);
                acc = cadd(acc, cmul(x[(a * Nb + b) * Nc + c], w));
            }
    y1[0] = acc.re; y1[1] = acc.im;
    free(Ta); free(Tb); free(Tc);
    return 0;
}
