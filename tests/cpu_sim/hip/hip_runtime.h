// Host emulation of the parts of the HIP device model that the nested-step
// kernels use, so that their device code can be compiled with a host C++
// compiler (and AddressSanitizer) and run on the CPU in tests.
//
// Model: every thread of a workgroup is a host thread; the blocks of a grid
// run one after another.  __syncthreads() is a barrier over the block's live
// threads, a wavefront shuffle is an exchange through a per-wavefront buffer
// between two barriers over the wavefront's live lanes, and a __shared__
// variable is a static (one block runs at a time).  A thread that returns
// leaves every barrier it belongs to, as an exited lane does on the device.
// A barrier or shuffle that not every live thread reaches (divergent code)
// stops the program with a message after a timeout instead of hanging.
//
// This header stands in for <hip/hip_runtime.h> only when the test harness
// puts this directory first on the include path; it is not part of the library.
#pragma once

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __shared__ static
#define __launch_bounds__(...)

struct alignas(16) double2 { double x, y; };
struct alignas(8) float2 { float x, y; };
inline double2 make_double2(double a, double b) { return double2{a, b}; }
inline float2 make_float2(float a, float b) { return float2{a, b}; }

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef int hipError_t;
enum { hipSuccess = 0 };

inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline unsigned int __float_as_uint(float f) { unsigned int u; memcpy(&u, &f, 4); return u; }
inline float __uint_as_float(unsigned int u) { float f; memcpy(&f, &u, 4); return f; }

namespace hipsim {

struct Idx { unsigned x = 0, y = 0, z = 0; };
inline thread_local Idx tidx, bidx, bdim;
inline thread_local int flat_tid = 0;

// Barrier over a changing set of live threads.  Arrivals are counted under a
// mutex; waiters spin on the generation number, yielding the core, which
// with hundreds of threads on a few cores is much faster than sleeping.
class Barrier {
  public:
    void reset(int n) { live_ = n; waiting_ = 0; }
    void wait(const char* what) {
        unsigned long g;
        {
            std::lock_guard<std::mutex> l(m_);
            g = gen_.load(std::memory_order_relaxed);
            if (++waiting_ == live_) { release(); return; }
        }
        const auto t0 = std::chrono::steady_clock::now();
        for (unsigned long spins = 1; gen_.load(std::memory_order_acquire) == g; ++spins) {
            std::this_thread::yield();
            if ((spins & 0xFFFF) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(300)) {
                fprintf(stderr, "hipsim: %s not reached by every live thread (%d of %d waiting)\n", what,
                        waiting_, live_);
                abort();
            }
        }
    }
    void leave() {
        std::lock_guard<std::mutex> l(m_);
        --live_;
        if (waiting_ > 0 && waiting_ == live_) release();
    }

  private:
    void release() { waiting_ = 0; gen_.fetch_add(1, std::memory_order_release); }
    std::mutex m_;
    int live_ = 0, waiting_ = 0;
    std::atomic<unsigned long> gen_{0};
};

struct Block {
    int nthreads = 0, nwaves = 0;
    Barrier block;
    std::vector<Barrier> waves;
    std::vector<uint64_t> xbuf;   // one word per lane
};
inline Block* g_block = nullptr;
inline int g_only_y = -1;   // >= 0: a launch runs only the blocks with blockIdx.y == g_only_y

inline void syncthreads() { g_block->block.wait("__syncthreads"); }

template <typename T>
inline T shfl(T v, int src) {
    static_assert(sizeof(T) <= 8, "shuffle of a word of at most 8 bytes");
    const int lane = flat_tid & 63, wave = flat_tid >> 6;
    Block& B = *g_block;
    uint64_t w = 0;
    memcpy(&w, &v, sizeof(T));
    B.xbuf[(size_t)wave * 64 + lane] = w;
    B.waves[wave].wait("wavefront shuffle");
    const int s = ((src % 64) + 64) % 64;
    const uint64_t r = B.xbuf[(size_t)wave * 64 + s];
    B.waves[wave].wait("wavefront shuffle");
    T out;
    memcpy(&out, &r, sizeof(T));
    return out;
}

template <typename... P, typename... A>
void launch(void (*kernel)(P...), dim3 grid, dim3 block, A... args) {
    const int nt = (int)(block.x * block.y * block.z);
    for (unsigned bz = 0; bz < grid.z; ++bz)
        for (unsigned by = 0; by < grid.y; ++by)
            for (unsigned bx = 0; bx < grid.x; ++bx) {
                if (g_only_y >= 0 && (int)by != g_only_y) continue;
                Block B;
                B.nthreads = nt;
                B.nwaves = (nt + 63) / 64;
                B.block.reset(nt);
                B.waves = std::vector<Barrier>(B.nwaves);
                for (int w = 0; w < B.nwaves; ++w) B.waves[w].reset(std::min(64, nt - 64 * w));
                B.xbuf.assign((size_t)B.nwaves * 64, 0);
                g_block = &B;
                std::vector<std::thread> th;
                th.reserve(nt);
                for (int t = 0; t < nt; ++t)
                    th.emplace_back([&, t] {
                        flat_tid = t;
                        tidx.x = t % block.x;
                        tidx.y = (t / block.x) % block.y;
                        tidx.z = t / (block.x * block.y);
                        bidx.x = bx; bidx.y = by; bidx.z = bz;
                        bdim.x = block.x; bdim.y = block.y; bdim.z = block.z;
                        kernel(args...);
                        B.waves[t >> 6].leave();
                        B.block.leave();
                    });
                for (auto& x : th) x.join();
                g_block = nullptr;
            }
}

}  // namespace hipsim

#define threadIdx (::hipsim::tidx)
#define blockIdx (::hipsim::bidx)
#define blockDim (::hipsim::bdim)
#define __syncthreads() ::hipsim::syncthreads()

template <typename T> inline T __shfl(T v, int src, int width = 64) { (void)width; return ::hipsim::shfl(v, src); }
template <typename T> inline T __shfl_xor(T v, int m, int width = 64) {
    (void)width;
    return ::hipsim::shfl(v, (::hipsim::flat_tid & 63) ^ m);
}

inline int atomicMax(int* a, int v) {
    int old = __atomic_load_n(a, __ATOMIC_SEQ_CST);
    while (old < v && !__atomic_compare_exchange_n(a, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return old;
}

#define hipLaunchKernelGGL(K, G, B, SH, ST, ...) ::hipsim::launch(K, G, B, ##__VA_ARGS__)
#define hipExtLaunchKernelGGL(K, G, B, SH, ST, EA, EB, FL, ...) ::hipsim::launch(K, G, B, ##__VA_ARGS__)
