// fft_kernel.hpp -- the stand-alone axis-pass kernel: one workgroup per tile
// of W lines (device body in fft_device.hpp).
#pragma once

#include "fft_device.hpp"

namespace offt {

// MAXT: the largest workgroup the kernel is compiled for (launch bound).
// P: the parts its LDS exchanges run in (P > 1: strided lines only).
template <typename V, int MAXT, int L, int TPL, int P, int... Rs>
__global__ void __launch_bounds__(MAXT) fft_pass_kernel(PassArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const int64_t l0 = xcd_tile(blockIdx.x, gridDim.x, a.xcd_remap) << a.logW;
    pass_tile_parts<V, L, TPL, P, Rs...>(a, lds, l0);
}

// Transposing pass (modes 2 and 3): one workgroup per tile of W lines.
template <typename V, int MAXT, int L, int TPL, int P, int... Rs>
__global__ void __launch_bounds__(MAXT) fft_tpass_kernel(PassArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const int64_t l0 = xcd_tile(blockIdx.x, gridDim.x, a.xcd_remap) << a.logW;
    pass_tile_transpose<V, L, TPL, P, Rs...>(a, lds, l0);
}

}  // namespace offt
