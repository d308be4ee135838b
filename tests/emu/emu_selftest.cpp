// Kernels with planted synchronisation mistakes, run only by the host
// emulation (never compiled for a GPU), to show that the emulator reports
// each kind of mistake it claims to detect.
#include <stdio.h>

#include "hip_emu.h"

namespace selftest {

// A persistent loop over tickets in which the threads of an empty item skip
// the barrier that the others wait at ("continue" around __syncthreads).
__global__ void k_continue_around_barrier(unsigned long long* ticket, const int* items, int n,
                                          int* out) {
    __shared__ unsigned long long t;
    for (;;) {
        if (threadIdx.x == 0) t = atomicAdd(ticket, 1ull);
        __syncthreads();
        const unsigned long long k = t;
        if (k >= (unsigned long long)n) break;
        if (items[k] == 0 && threadIdx.x % 2) continue;  // planted: not uniform
        __syncthreads();
        if (threadIdx.x == 0) out[k] = items[k];
    }
}

// Some threads return before a barrier that the rest of the workgroup waits at.
__global__ void k_return_before_barrier(int* out) {
    __shared__ int s;
    if (threadIdx.x >= 32) return;  // planted
    if (threadIdx.x == 0) s = 1;
    __syncthreads();
    out[threadIdx.x] = s;
}

// A workgroup waits for a flag that only a later workgroup sets.
__global__ void k_wait_for_later_block(int* flag, int* out) {
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            int spins = 0;
            while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                   ++spins < (1 << 21))
                __builtin_amdgcn_s_sleep(1);
            out[0] = spins;
        }
    } else if (threadIdx.x == 0) {
        __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// A barrier inside a branch that depends on the thread: half the workgroup
// takes a different barrier.
__global__ void k_barrier_in_branch(int* out) {
    __shared__ int s[64];
    s[threadIdx.x] = (int)threadIdx.x;
    if (threadIdx.x < 16) {
        __syncthreads();  // planted
        out[threadIdx.x] = s[63 - threadIdx.x];
    } else {
        __syncthreads();
        out[threadIdx.x] = s[threadIdx.x];
    }
}

}  // namespace selftest

extern "C" const char* emu_errors();
extern "C" void emu_clear_errors();

int emu_selftest(FILE* out) {
    using namespace selftest;
    auto report = [&](const char* name) {
        fprintf(out, "%s: %s\n", name, emu_errors()[0] ? "reported" : "NOT REPORTED");
        fprintf(out, "%s", emu_errors());
        emu_clear_errors();
    };
    static unsigned long long ticket = 0;
    static int items[4] = {1, 0, 1, 1}, res[64], flag = 0;
    hipLaunchKernelGGL(k_continue_around_barrier, dim3(1), dim3(64), 0, 0, &ticket, items, 4, res);
    report("continue_around_barrier");
    hipLaunchKernelGGL(k_return_before_barrier, dim3(1), dim3(64), 0, 0, res);
    report("return_before_barrier");
    hipLaunchKernelGGL(k_wait_for_later_block, dim3(2), dim3(64), 0, 0, &flag, res);
    report("wait_for_later_block");
    hipLaunchKernelGGL(k_barrier_in_branch, dim3(1), dim3(64), 0, 0, res);
    report("barrier_in_branch");
    return 0;
}
