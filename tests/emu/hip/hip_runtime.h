// Test infrastructure: the subset of the HIP device language and runtime that the library's
// kernels use, on the host, so the same kernel sources run on the CPU under AddressSanitizer.
//
// Every block of a launch runs on its own, one after another; each thread of a block is a
// coroutine.  A thread runs until it reaches a wave operation (ballot, shuffle, wave barrier)
// or __syncthreads(); a wave operation completes once every thread of the wave that has not
// returned waits at it (threads that returned are inactive lanes, as on the device), a block
// barrier once every thread of the block that has not returned waits at it.  Wave operations
// of one wave waiting at different call sites are reported as an error (divergent lanes).
// LDS arrays declared in a kernel are function-scope statics, shared by the blocks of a
// launch in turn; the dynamic LDS of a launch is one buffer of the launch's size.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>
#include <type_traits>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

struct dim3 {
    uint32_t x, y, z;
    constexpr dim3(uint32_t x_ = 1, uint32_t y_ = 1, uint32_t z_ = 1) : x(x_), y(y_), z(z_) {}
};

namespace emu {

struct Lane;
Lane* cur();
const dim3& thread_idx();
const dim3& block_idx();
const dim3& block_dim();
const dim3& grid_dim();
void* dyn_lds();

enum Op : int { kOpShfl = 1, kOpShflUp, kOpShflDown, kOpShflXor, kOpBallot, kOpWaveBarrier };
// Deposits this lane's operand of a wave operation, waits for the wave, returns the result.
uint64_t wave_op(int op, uint64_t bits, int param, int width, const void* site);
void sync_block(const void* site);

template <typename T>
inline uint64_t to_bits(T v)
{
    static_assert(sizeof(T) <= 8 && std::is_trivially_copyable<T>::value, "wave operand");
    uint64_t b = 0;
    std::memcpy(&b, &v, sizeof(T));
    return b;
}
template <typename T>
inline T from_bits(uint64_t b)
{
    T v;
    std::memcpy(&v, &b, sizeof(T));
    return v;
}

void launch(const dim3& grid, const dim3& block, size_t dyn_lds_bytes,
            const std::function<void()>& body);
// Fills a kernel's static LDS array with a byte pattern the first time a thread of the running
// block reaches its declaration.
void lds_fresh(void* p, size_t bytes);

}  // namespace emu

#define threadIdx (::emu::thread_idx())
#define blockIdx (::emu::block_idx())
#define blockDim (::emu::block_dim())
#define gridDim (::emu::grid_dim())

__attribute__((noinline)) inline void __syncthreads() { ::emu::sync_block(__builtin_return_address(0)); }

template <typename T>
__attribute__((noinline)) T __shfl(T v, int src, int width = 64)
{
    return ::emu::from_bits<T>(::emu::wave_op(::emu::kOpShfl, ::emu::to_bits(v), src, width,
                                              __builtin_return_address(0)));
}
template <typename T>
__attribute__((noinline)) T __shfl_up(T v, unsigned int d, int width = 64)
{
    return ::emu::from_bits<T>(::emu::wave_op(::emu::kOpShflUp, ::emu::to_bits(v), (int)d, width,
                                              __builtin_return_address(0)));
}
template <typename T>
__attribute__((noinline)) T __shfl_down(T v, unsigned int d, int width = 64)
{
    return ::emu::from_bits<T>(::emu::wave_op(::emu::kOpShflDown, ::emu::to_bits(v), (int)d,
                                              width, __builtin_return_address(0)));
}
template <typename T>
__attribute__((noinline)) T __shfl_xor(T v, int m, int width = 64)
{
    return ::emu::from_bits<T>(::emu::wave_op(::emu::kOpShflXor, ::emu::to_bits(v), m, width,
                                              __builtin_return_address(0)));
}
__attribute__((noinline)) inline unsigned long long __ballot(int pred)
{
    return ::emu::wave_op(::emu::kOpBallot, pred ? 1u : 0u, 0, 64, __builtin_return_address(0));
}
__attribute__((noinline)) inline void emu_wave_barrier()
{
    ::emu::wave_op(::emu::kOpWaveBarrier, 0, 0, 64, __builtin_return_address(0));
}
#define __builtin_amdgcn_wave_barrier() emu_wave_barrier()
// one thread runs at a time: fences order nothing further
#define __builtin_amdgcn_fence(...) ((void)0)

using std::isfinite;
using std::isinf;
using std::isnan;

template <typename A, typename B>
inline typename std::common_type<A, B>::type min(A a, B b)
{
    using T = typename std::common_type<A, B>::type;
    return (T)a < (T)b ? (T)a : (T)b;
}
template <typename A, typename B>
inline typename std::common_type<A, B>::type max(A a, B b)
{
    using T = typename std::common_type<A, B>::type;
    return (T)a > (T)b ? (T)a : (T)b;
}

inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }

inline double __dmul_rn(double a, double b) { return a * b; }
inline double __ddiv_rn(double a, double b) { return a / b; }
inline double __dadd_rn(double a, double b) { return a + b; }

// The hardware's transcendental instructions: log base 2, and sine / cosine of an angle given
// in revolutions.
inline float emu_log2f(float x) { return std::log2(x); }
inline float emu_sinrevf(float x) { return (float)std::sin(6.283185307179586 * (double)x); }
inline float emu_cosrevf(float x) { return (float)std::cos(6.283185307179586 * (double)x); }
#define __builtin_amdgcn_logf(x) emu_log2f(x)
#define __builtin_amdgcn_sqrtf(x) std::sqrt((float)(x))
#define __builtin_amdgcn_sinf(x) emu_sinrevf(x)
#define __builtin_amdgcn_cosf(x) emu_cosrevf(x)

// one thread runs at a time: atomics are plain read-modify-writes
inline uint32_t atomicOr(uint32_t* p, uint32_t v) { const uint32_t o = *p; *p = o | v; return o; }
inline uint32_t atomicAdd(uint32_t* p, uint32_t v) { const uint32_t o = *p; *p = o + v; return o; }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v)
{
    const unsigned long long o = *p;
    *p = o + v;
    return o;
}

struct uint4 {
    uint32_t x, y, z, w;
};
inline uint4 make_uint4(uint32_t x, uint32_t y, uint32_t z, uint32_t w) { return {x, y, z, w}; }

// ---- runtime ------------------------------------------------------------------------------
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorInvalidSymbol = 13,
    hipErrorLaunchFailure = 719,
};
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };

namespace emu {
hipError_t& last_error();
}
inline hipError_t hipGetLastError()
{
    const hipError_t e = ::emu::last_error();
    ::emu::last_error() = hipSuccess;
    return e;
}
inline const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated HIP error"; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
#define HIP_SYMBOL(x) ((const void*)&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym)
{
    *p = const_cast<void*>(sym);
    return hipSuccess;
}

#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) \
    ::emu::launch(dim3(grid), dim3(block), (size_t)(lds), [=]() { kernel(__VA_ARGS__); })
