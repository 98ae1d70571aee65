// twiddle.hip -- twiddle tables W_L^m = exp(-2 pi i m / L), m < L, generated on
// the GPU in binary64 and rounded to nearest for the binary32 path.
//
// Argument reduction is exact integer arithmetic: with 4m = q L + r
// (0 <= r < L) the angle is (pi/2) (q + r/L).  The in-quadrant angle
// phi = (pi/2) r/L is evaluated as sinpi/cospi of r/(2L) when 2r <= L, and as
// the complementary angle otherwise, so the argument of sinpi/cospi never
// exceeds 1/4; then (cos, sin) is rotated by q quarter turns.  Values at the
// quarter points (r = 0) are exactly 1, -i, -1, +i.
#include <algorithm>

#include "offt_internal.h"

namespace offt {

__device__ inline void unit_root(int64_t m, int64_t n, double* c, double* s) {
    const int64_t m4 = 4 * (m % n);
    const int64_t q = m4 / n;
    const int64_t r = m4 - q * n;
    double cp, sp;
    if (2 * r <= n) {
        const double x = (double)r / (double)(2 * n);
        sincospi(x, &sp, &cp);
    } else {
        const double x = (double)(n - r) / (double)(2 * n);
        sincospi(x, &cp, &sp);   // cos(phi) = sin(pi/2 - phi), sin(phi) = cos(pi/2 - phi)
    }
    // rotate (cp, sp) by q quarter turns: (c, s) -> (-s, c)
    for (int k = 0; k < (int)q; ++k) {
        const double t = cp;
        cp = -sp;
        sp = t;
    }
    *c = cp;
    *s = sp;
}

template <typename V>
__global__ void twiddle_kernel(V* __restrict__ out, int64_t n) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double c, s;
    unit_root(m, n, &c, &s);
    V v;
    v.x = (decltype(v.x))c;     // round to nearest for binary32
    v.y = (decltype(v.y))(-s);  // forward sign
    out[m] = v;
}

hipError_t launch_twiddles(void* out, int64_t n, int dtype, hipStream_t s) {
    const int threads = 256;
    const unsigned blocks = (unsigned)((n + threads - 1) / threads);
    if (dtype == 0)
        hipLaunchKernelGGL(twiddle_kernel<double2>, dim3(blocks), dim3(threads), 0, s,
                           static_cast<double2*>(out), n);
    else
        hipLaunchKernelGGL(twiddle_kernel<float2>, dim3(blocks), dim3(threads), 0, s,
                           static_cast<float2*>(out), n);
    return hipGetLastError();
}

// Tuning data: n reals (two per complex element) uniform in [-1, 1) from a
// SplitMix64-style hash of (index, key).  Timings on all-zero buffers are not
// representative: on this device's HBM a copy of zeros moves far more bytes
// per second than a copy of random values.
template <typename S>
__global__ void fill_uniform_kernel(S* __restrict__ out, int64_t n, uint64_t key) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = key + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        out[i] = (S)((double)(z >> 11) * 0x1.0p-52 - 1.0);
    }
}

hipError_t launch_fill_uniform(void* out, int64_t nelem, int dtype, uint64_t key, hipStream_t s) {
    const int threads = 256;
    const int64_t n = 2 * nelem;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + threads - 1) / threads, 8192);
    if (n <= 0) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL(fill_uniform_kernel<double>, dim3(blocks), dim3(threads), 0, s,
                           static_cast<double*>(out), n, key);
    else
        hipLaunchKernelGGL(fill_uniform_kernel<float>, dim3(blocks), dim3(threads), 0, s,
                           static_cast<float*>(out), n, key);
    return hipGetLastError();
}

}  // namespace offt
