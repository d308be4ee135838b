// Host emulation of the subset of HIP that libtpx's kernels and C-ABI layer
// use, for CPU checks of the kernels (test infrastructure, never linked into
// the library).  The kernel sources are compiled unchanged by g++ with this
// header force-included.
//
// Execution model:
//   * a launch runs its workgroups one after another, in block order;
//   * the threads of a workgroup are cooperative fibers (ucontext) on one OS
//     thread, so every read-modify-write is atomic by construction;
//   * __syncthreads and its reductions are counting barriers: a barrier opens
//     only when every thread of the workgroup has arrived at the same barrier
//     call (same call site, same occurrence).  A thread that arrives at a
//     different barrier, or that has exited while others wait, is reported as
//     a divergent barrier; a state where no thread can run is a deadlock;
//   * cross-lane operations (__shfl*, __ballot, readfirstlane) synchronise the
//     64 lanes of a wave: they complete once no lane of the wave can run any
//     further, over the lanes that reached the same call (the active lanes),
//     which is how a wave executes them under an execution mask;
//   * atomics and the scoped atomic loads and stores may hand the processor
//     to another thread (seeded, probability EMU_PREEMPT per mille), so that
//     runs explore different interleavings;
//   * device memory is host memory (malloc), so AddressSanitizer checks every
//     global access; __shared__ arrays are static storage, checked the same
//     way for overruns.
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <type_traits>

// ------------------------------------------------------------ qualifiers
#define __global__
#define __device__
#define __align__(n) alignas(n)
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
// per-kernel occupancy hints of the AMDGPU back end: nothing to emulate
#define amdgpu_waves_per_eu(...)
#define __shared__ static

// ------------------------------------------------------------ vector types
struct dim3 {
    uint32_t x, y, z;
    constexpr dim3(uint32_t x_ = 1, uint32_t y_ = 1, uint32_t z_ = 1) : x(x_), y(y_), z(z_) {}
};
struct uint4 {
    uint32_t x, y, z, w;
};
struct uint2 {
    uint32_t x, y;
};
inline uint4 make_uint4(uint32_t x, uint32_t y, uint32_t z, uint32_t w) { return uint4{x, y, z, w}; }
inline uint2 make_uint2(uint32_t x, uint32_t y) { return uint2{x, y}; }

// ------------------------------------------------------------ runtime types
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 };
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
typedef int hipMemcpyKind;
enum {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
};
enum { hipStreamDefault = 0, hipStreamNonBlocking = 1 };
enum { hipEventDefault = 0, hipEventDisableTiming = 2 };
enum { hipHostMallocDefault = 0 };

#define __HIP_MEMORY_SCOPE_WAVEFRONT 2
#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#define __HIP_MEMORY_SCOPE_AGENT 4
#define __HIP_MEMORY_SCOPE_SYSTEM 5

namespace emu {

struct Thread {
    dim3 tid;
    dim3 bid;
    uint32_t flat;  // flat thread index in the workgroup
};
extern Thread* cur;
extern dim3 grid_dim, block_dim;

void launch(dim3 grid, dim3 block, const std::function<void()>& body);
void syncthreads(uintptr_t site);
int syncthreads_red(uintptr_t site, int kind, int v);  // 0: or, 1: and, 2: count
uint64_t wave_op(uintptr_t site, int kind, uint64_t v, int arg);
void maybe_preempt();
void yield_sleep();
void note_error(const char* what);

enum { kShflXor = 0, kShflUp = 1, kShflDown = 2, kShfl = 3, kBallot = 4, kFirst = 5, kDpp = 6 };

template <class T>
inline uint64_t to_bits(T v) {
    uint64_t b = 0;
    memcpy(&b, &v, sizeof(T));
    return b;
}
template <class T>
inline T from_bits(uint64_t b) {
    T v;
    memcpy(&v, &b, sizeof(T));
    return v;
}

}  // namespace emu

#define EMU_SITE ((uintptr_t)__builtin_return_address(0))

inline const dim3& emu_tidx() { return emu::cur->tid; }
inline const dim3& emu_bidx() { return emu::cur->bid; }
#define threadIdx emu_tidx()
#define blockIdx emu_bidx()
#define blockDim emu::block_dim
#define gridDim emu::grid_dim

__attribute__((noinline)) inline void __syncthreads() { emu::syncthreads(EMU_SITE); }
__attribute__((noinline)) inline int __syncthreads_or(int p) {
    return emu::syncthreads_red(EMU_SITE, 0, p != 0);
}
__attribute__((noinline)) inline int __syncthreads_and(int p) {
    return emu::syncthreads_red(EMU_SITE, 1, p != 0);
}
__attribute__((noinline)) inline int __syncthreads_count(int p) {
    return emu::syncthreads_red(EMU_SITE, 2, p != 0);
}
inline void __threadfence() {}
inline void __threadfence_block() {}

inline unsigned __lane_id() { return emu::cur->flat & 63u; }

template <class T>
__attribute__((noinline)) T __shfl_xor(T v, int m, int w = 64) {
    (void)w;
    return emu::from_bits<T>(emu::wave_op(EMU_SITE, emu::kShflXor, emu::to_bits(v), m));
}
template <class T>
__attribute__((noinline)) T __shfl_up(T v, unsigned d, int w = 64) {
    (void)w;
    return emu::from_bits<T>(emu::wave_op(EMU_SITE, emu::kShflUp, emu::to_bits(v), (int)d));
}
template <class T>
__attribute__((noinline)) T __shfl_down(T v, unsigned d, int w = 64) {
    (void)w;
    return emu::from_bits<T>(emu::wave_op(EMU_SITE, emu::kShflDown, emu::to_bits(v), (int)d));
}
template <class T>
__attribute__((noinline)) T __shfl(T v, int src, int w = 64) {
    (void)w;
    return emu::from_bits<T>(emu::wave_op(EMU_SITE, emu::kShfl, emu::to_bits(v), src));
}
__attribute__((noinline)) inline unsigned long long __ballot(int p) {
    return emu::wave_op(EMU_SITE, emu::kBallot, p != 0, 0);
}
template <class T>
__attribute__((noinline)) T emu_readfirstlane(T v) {
    return emu::from_bits<T>(emu::wave_op(EMU_SITE, emu::kFirst, emu::to_bits(v), 0));
}
#define __builtin_amdgcn_readfirstlane(v) emu_readfirstlane(v)
// DPP move (the controls the kernels use: row_shr:n, wave_shr:1,
// row_bcast:15, row_bcast:31); the wave op returns the source lane's value,
// or bit 32 set when the lane has no active source lane
__attribute__((noinline)) inline int emu_update_dpp(int old, int src, int ctrl, int row_mask,
                                                    int bank_mask, bool bound_ctrl) {
    const uint64_t r = emu::wave_op(EMU_SITE, emu::kDpp, (uint32_t)src, ctrl);
    const unsigned l = __lane_id();
    if (!((row_mask >> (l >> 4)) & 1) || !((bank_mask >> ((l >> 2) & 3)) & 1)) return old;
    if (r >> 32) return bound_ctrl ? 0 : old;
    return (int)(uint32_t)r;
}
#define __builtin_amdgcn_update_dpp(o, s, c, rm, bm, bc) emu_update_dpp(o, s, c, rm, bm, bc)
#define __builtin_amdgcn_s_sleep(n) emu::yield_sleep()
#define __builtin_amdgcn_wave_barrier() ((void)0)
#define __builtin_nontemporal_load(p) (*(p))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))

inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __popc(unsigned v) { return __builtin_popcount(v); }
inline int __ffsll(unsigned long long v) { return __builtin_ffsll((long long)v); }
inline int __ffs(unsigned v) { return __builtin_ffs((int)v); }
inline int __clzll(unsigned long long v) { return v ? __builtin_clzll(v) : 64; }
inline int __clz(unsigned v) { return v ? __builtin_clz(v) : 32; }

template <class A, class B>
inline typename std::common_type<A, B>::type min(A a, B b) {
    typedef typename std::common_type<A, B>::type C;
    return (C)a < (C)b ? (C)a : (C)b;
}
template <class A, class B>
inline typename std::common_type<A, B>::type max(A a, B b) {
    typedef typename std::common_type<A, B>::type C;
    return (C)a > (C)b ? (C)a : (C)b;
}

// ------------------------------------------------------------ atomics
template <class T>
inline T atomicAdd(T* p, T v) {
    emu::maybe_preempt();
    const T o = *p;
    *p = o + v;
    return o;
}
inline unsigned long long atomicAdd(unsigned long long* p, uint64_t v) {
    return atomicAdd<unsigned long long>(p, (unsigned long long)v);
}
inline unsigned atomicAdd(unsigned* p, int v) { return atomicAdd<unsigned>(p, (unsigned)v); }
template <class T>
inline T atomicSub(T* p, T v) {
    emu::maybe_preempt();
    const T o = *p;
    *p = o - v;
    return o;
}
template <class T>
inline T atomicOr(T* p, T v) {
    emu::maybe_preempt();
    const T o = *p;
    *p = o | v;
    return o;
}
template <class T>
inline T atomicAnd(T* p, T v) {
    emu::maybe_preempt();
    const T o = *p;
    *p = o & v;
    return o;
}
template <class T>
inline T atomicMin(T* p, T v) {
    emu::maybe_preempt();
    const T o = *p;
    *p = v < o ? v : o;
    return o;
}
inline unsigned long long atomicMin(unsigned long long* p, uint64_t v) {
    return atomicMin<unsigned long long>(p, (unsigned long long)v);
}
template <class T>
inline T atomicMax(T* p, T v) {
    emu::maybe_preempt();
    const T o = *p;
    *p = v > o ? v : o;
    return o;
}
inline unsigned long long atomicMax(unsigned long long* p, uint64_t v) {
    return atomicMax<unsigned long long>(p, (unsigned long long)v);
}
template <class T>
inline T atomicExch(T* p, T v) {
    emu::maybe_preempt();
    const T o = *p;
    *p = v;
    return o;
}
template <class T>
inline T atomicCAS(T* p, T expect, T v) {
    emu::maybe_preempt();
    const T o = *p;
    if (o == expect) *p = v;
    return o;
}

template <class T>
inline T __hip_atomic_load(const T* p, int order, int scope) {
    (void)order;
    (void)scope;
    emu::maybe_preempt();
    return *p;
}
template <class T, class V>
inline void __hip_atomic_store(T* p, V v, int order, int scope) {
    (void)order;
    (void)scope;
    emu::maybe_preempt();
    *p = (T)v;
}
template <class T, class V>
inline T __hip_atomic_fetch_add(T* p, V v, int order, int scope) {
    (void)order;
    (void)scope;
    return atomicAdd(p, (T)v);
}
template <class T, class V>
inline T __hip_atomic_fetch_max(T* p, V v, int order, int scope) {
    (void)order;
    (void)scope;
    return atomicMax(p, (T)v);
}
template <class T, class V>
inline bool __hip_atomic_compare_exchange_strong(T* p, T* expect, V v, int o1, int o2, int scope) {
    (void)o1;
    (void)o2;
    (void)scope;
    emu::maybe_preempt();
    if (*p == *expect) {
        *p = (T)v;
        return true;
    }
    *expect = *p;
    return false;
}

// ------------------------------------------------------------ runtime calls
hipError_t hipMalloc(void** p, size_t n);
template <class T>
inline hipError_t hipMalloc(T** p, size_t n) {
    return hipMalloc((void**)p, n);
}
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags = 0);
template <class T>
inline hipError_t hipHostMalloc(T** p, size_t n, unsigned flags = 0) {
    return hipHostMalloc((void**)p, n, flags);
}
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st = 0);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st = 0);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = 0);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetLastError();
hipError_t hipPeekAtLastError();
hipError_t hipDeviceSynchronize();
hipError_t hipGetDevice(int* d);
hipError_t hipSetDevice(int d);
enum { hipDeviceAttributeMultiprocessorCount = 1 };
// a small device: persistent grids take several work items per workgroup
hipError_t hipDeviceGetAttribute(int* v, int attr, int dev);
// a file-scope device array is an ordinary host array here: its symbol is
// its address
#define HIP_SYMBOL(x) ((const void*)&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
    *p = const_cast<void*>(sym);
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t e);

#define hipLaunchKernelGGL(K, G, B, SH, ST, ...) \
    ::emu::launch(dim3(G), dim3(B), [=]() { K(__VA_ARGS__); })
