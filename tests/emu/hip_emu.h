// hip_emu.h -- just enough of HIP to compile the library's device headers
// (fft_device.hpp, many_device.hpp) as host C++ and run one workgroup on CPU
// threads.  Test infrastructure: it lets the tile code be run under
// AddressSanitizer and with a barrier that detects threads reaching
// different numbers of __syncthreads().
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) alignas(n)

struct float2 { float x, y; };
struct double2 { double x, y; };

struct EmuDim { unsigned x = 0, y = 0, z = 0; };
extern thread_local EmuDim threadIdx;
extern EmuDim blockIdx, blockDim, gridDim;

// Barrier for the emulated workgroup; reports a mismatch instead of hanging.
struct EmuBarrier {
    std::mutex m;
    std::condition_variable cv;
    int n = 0, waiting = 0;
    long generation = 0;
    bool broken = false;
    void reset(int threads) { n = threads; waiting = 0; generation = 0; broken = false; }
    void arrive_and_wait() {
        std::unique_lock<std::mutex> lk(m);
        if (broken) return;
        const long gen = generation;
        if (++waiting == n) {
            waiting = 0;
            ++generation;
            cv.notify_all();
            return;
        }
        if (!cv.wait_for(lk, std::chrono::seconds(180), [&] { return generation != gen || broken; })) {
            broken = true;
            std::fprintf(stderr, "EMU: barrier mismatch: %d of %d threads waiting at generation %ld\n", waiting, n,
                         gen);
            cv.notify_all();
        }
    }
};
extern EmuBarrier g_emu_barrier;
extern thread_local long g_emu_barrier_count;

inline void __syncthreads() {
    ++g_emu_barrier_count;
    g_emu_barrier.arrive_and_wait();
}

#define __HIP_MEMORY_SCOPE_AGENT 1
#define __hip_atomic_fetch_add(p, v, o, s) __atomic_fetch_add((p), (v), (o))
#define __hip_atomic_load(p, o, s) __atomic_load_n((p), (o))
#define __hip_atomic_store(p, v, o, s) __atomic_store_n((p), (v), (o))
#define __builtin_amdgcn_fence(o, scope) __atomic_thread_fence(o)
#define __builtin_amdgcn_s_sleep(n) std::this_thread::sleep_for(std::chrono::microseconds(20))
#define __builtin_amdgcn_s_waitcnt(n) ((void)0)
// A value made opaque to the device compiler's loop hoisting: nothing to do on the host.
#define OFFT_OPAQUE_VGPR(x) ((void)(x))
// One emulated thread per wavefront: a wave-uniform value is the thread's own.
#define __builtin_amdgcn_readfirstlane(x) (x)

// Streaming (non-temporal) accesses are ordinary accesses on the host.
#define __builtin_nontemporal_load(p) (*(p))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))
