// Host emulation runtime for libtpx's kernels (test infrastructure).  See
// hip_emu.h for the execution model.
#include "hip_emu.h"

#include <stdio.h>
#include <stdlib.h>
#include <sys/mman.h>

#include <random>
#include <string>
#include <vector>

#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#else
#define EMU_ASAN 0
#endif

namespace emu {

Thread* cur = nullptr;
dim3 grid_dim, block_dim;

namespace {

enum State { kReady, kAtBarrier, kAtWave, kExited };

constexpr size_t kStack = 256 * 1024;
constexpr int kMaxThreads = 1024;

// Minimal x86-64 context switch: saves the callee-saved registers on the
// current stack, stores the stack pointer in *save and continues on the stack
// `next` (a stack saved by an earlier switch, or a fresh one laid out by
// fresh_stack).  Far cheaper than swapcontext, which makes a system call.
extern "C" void emu_ctx_switch(void** save, void* next);
asm(R"(
.text
.globl emu_ctx_switch
.type emu_ctx_switch,@function
emu_ctx_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
.size emu_ctx_switch, .-emu_ctx_switch
)");

struct Fiber {
    void* sp = nullptr;
    char* stack = nullptr;
    State st = kExited;
    Thread th;
    // barrier
    uintptr_t site = 0;
    uint64_t nbar = 0;  // barriers passed so far
    int red_kind = -1, red_v = 0, red_out = 0;
    // wave operation
    int wkind = 0, warg = 0;
    uint64_t wv = 0, wout = 0;
    void* fake = nullptr;
};

void* sched_sp = nullptr;
const void* sched_bottom = nullptr;
size_t sched_size = 0;
void* sched_fake = nullptr;
Fiber fibers[kMaxThreads];
Fiber* running = nullptr;
int nthreads = 0;
const std::function<void()>* body_fn = nullptr;
std::mt19937_64 rng(12345);
int preempt_permille = 0;
uint64_t sleep_yields = 0;
std::string errors;
uint64_t n_launches = 0, n_blocks = 0, n_barriers = 0, n_wave_ops = 0, n_preempts = 0;
bool abandon = false;  // the current block deadlocked: its fibers are dropped

void add_error(const std::string& s) {
    if (errors.size() < 4096) errors += s + "\n";
}

[[noreturn]] void fiber_main() {
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &sched_bottom, &sched_size);
#endif
    (*body_fn)();
    running->st = kExited;
#if EMU_ASAN
    __sanitizer_start_switch_fiber(nullptr, sched_bottom, sched_size);
#endif
    void* dead;
    emu_ctx_switch(&dead, sched_sp);
    __builtin_unreachable();
}

// a fresh stack whose first switch lands in fiber_main
void* fresh_stack(char* stack) {
    uintptr_t top = ((uintptr_t)(stack + kStack)) & ~(uintptr_t)15;
    uintptr_t ret = top - 16;  // return-address slot, 16-byte aligned
    void** p = (void**)ret;
    p[0] = (void*)&fiber_main;
    for (int k = 1; k <= 6; ++k) p[-k] = nullptr;  // rbp, rbx, r12-r15
    return (void*)(ret - 48);
}

// hands the processor back to the scheduler; returns when resumed
void to_scheduler() {
    Fiber* f = running;
#if EMU_ASAN
    __sanitizer_start_switch_fiber(&f->fake, sched_bottom, sched_size);
#endif
    emu_ctx_switch(&f->sp, sched_sp);
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(f->fake, &sched_bottom, &sched_size);
#endif
    cur = &running->th;
}

void resume(Fiber* f) {
    running = f;
    cur = &f->th;
#if EMU_ASAN
    __sanitizer_start_switch_fiber(&sched_fake, f->stack, kStack);
#endif
    emu_ctx_switch(&sched_sp, f->sp);
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(sched_fake, nullptr, nullptr);
#endif
    running = nullptr;
}

// completes the wave operation of the lanes of wave w waiting at `site`
void release_wave(int w, uintptr_t site) {
    const int lo = w * 64, hi = std::min(nthreads, lo + 64);
    uint64_t active = 0;
    for (int i = lo; i < hi; ++i)
        if (fibers[i].st == kAtWave && fibers[i].site == site) active |= 1ull << (i - lo);
    ++n_wave_ops;
    const uint64_t poison = 0xDEADBEEFDEADBEEFull;
    auto val = [&](int l) -> uint64_t {
        return (l >= 0 && l < 64 && ((active >> l) & 1)) ? fibers[lo + l].wv : poison;
    };
    uint64_t ballot = 0;
    for (int i = lo; i < hi; ++i)
        if ((active >> (i - lo)) & 1)
            if (fibers[i].wv) ballot |= 1ull << (i - lo);
    int first = active ? __builtin_ctzll(active) : 0;
    for (int i = lo; i < hi; ++i) {
        if (!((active >> (i - lo)) & 1)) continue;
        Fiber& f = fibers[i];
        const int l = i - lo;
        switch (f.wkind) {
            case kShflXor: f.wout = val(l ^ f.warg); break;
            case kShflUp: f.wout = l - f.warg >= 0 ? val(l - f.warg) : f.wv; break;
            case kShflDown: f.wout = l + f.warg < 64 ? val(l + f.warg) : f.wv; break;
            case kShfl: f.wout = val(f.warg & 63); break;
            case kBallot: f.wout = ballot; break;
            case kFirst: f.wout = fibers[lo + first].wv; break;
            case kDpp: {
                const int c = f.warg;
                int src = -1;
                if (c > 0x110 && c <= 0x11F) {
                    if ((l & 15) >= c - 0x110) src = l - (c - 0x110);
                } else if (c == 0x138) {
                    if (l >= 1) src = l - 1;
                } else if (c == 0x142) {
                    if (l >= 16) src = (l & ~15) - 1;
                } else if (c == 0x143) {
                    if (l >= 32) src = 31;
                } else {
                    add_error("unsupported DPP control " + std::to_string(c));
                }
                f.wout = (src >= 0 && ((active >> src) & 1)) ? (fibers[lo + src].wv & 0xFFFFFFFFull)
                                                            : (1ull << 32);
                break;
            }
        }
        f.st = kReady;
    }
}

void run_block() {
    for (int i = 0; i < nthreads; ++i) {
        Fiber& f = fibers[i];
        f.sp = fresh_stack(f.stack);
        f.st = kReady;
        f.nbar = 0;
        f.fake = nullptr;
    }
    std::vector<int> ready;
    for (;;) {
        ready.clear();
        for (int i = 0; i < nthreads; ++i)
            if (fibers[i].st == kReady) ready.push_back(i);
        if (!ready.empty()) {
            if (preempt_permille > 0) {
                // random order among the runnable threads
                for (size_t k = ready.size(); k > 1; --k) {
                    const size_t j = rng() % k;
                    std::swap(ready[k - 1], ready[j]);
                }
            }
            for (int i : ready)
                if (fibers[i].st == kReady) resume(&fibers[i]);
            continue;
        }
        // nothing runnable: complete a wave operation if one is pending
        bool released = false;
        for (int w = 0; w * 64 < nthreads && !released; ++w) {
            uintptr_t site = 0;
            for (int i = w * 64; i < std::min(nthreads, w * 64 + 64); ++i)
                if (fibers[i].st == kAtWave) {
                    site = fibers[i].site;
                    break;
                }
            if (site) {
                release_wave(w, site);
                released = true;
            }
        }
        if (released) continue;
        int n_exit = 0, n_bar = 0;
        for (int i = 0; i < nthreads; ++i) {
            n_exit += fibers[i].st == kExited;
            n_bar += fibers[i].st == kAtBarrier;
        }
        if (n_exit == nthreads) return;
        // every live thread waits at a barrier
        char buf[256];
        if (n_exit > 0) {
            snprintf(buf, sizeof buf, "%d threads wait at a barrier while %d have exited", n_bar,
                     n_exit);
            add_error(buf);
            abandon = true;
            return;
        }
        const uintptr_t s0 = fibers[0].site;
        const uint64_t b0 = fibers[0].nbar;
        for (int i = 1; i < nthreads; ++i)
            if (fibers[i].site != s0 || fibers[i].nbar != b0) {
                snprintf(buf, sizeof buf,
                         "divergent barrier: thread 0 at site %#lx (barrier %lu), thread %d at "
                         "site %#lx (barrier %lu)",
                         (unsigned long)s0, (unsigned long)b0, i, (unsigned long)fibers[i].site,
                         (unsigned long)fibers[i].nbar);
                add_error(buf);
                abandon = true;
                return;
            }
        int red = fibers[0].red_kind == 1 ? 1 : 0;
        for (int i = 0; i < nthreads; ++i) {
            const Fiber& f = fibers[i];
            if (f.red_kind == 0) red |= f.red_v;
            if (f.red_kind == 1) red &= f.red_v;
            if (f.red_kind == 2) red += f.red_v;
        }
        ++n_barriers;
        for (int i = 0; i < nthreads; ++i) {
            fibers[i].red_out = red;
            fibers[i].st = kReady;
            fibers[i].nbar++;
        }
    }
}

}  // namespace

void launch(dim3 grid, dim3 block, const std::function<void()>& body) {
    static bool init = false;
    if (!init) {
        for (int i = 0; i < kMaxThreads; ++i) {
            void* p = mmap(nullptr, kStack, PROT_READ | PROT_WRITE,
                           MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
            if (p == MAP_FAILED) {
                fprintf(stderr, "emu: stack mmap failed\n");
                abort();
            }
            fibers[i].stack = (char*)p;
        }
        const char* pp = getenv("EMU_PREEMPT");
        preempt_permille = pp ? atoi(pp) : 0;
        const char* sd = getenv("EMU_SEED");
        rng.seed(sd ? strtoull(sd, nullptr, 10) : 12345);
        init = true;
    }
    const uint64_t nt = (uint64_t)block.x * block.y * block.z;
    if (nt == 0 || nt > (uint64_t)kMaxThreads) {
        add_error("launch with an invalid workgroup size");
        return;
    }
    ++n_launches;
    static const bool trace = getenv("EMU_TRACE") != nullptr;
    if (trace) fprintf(stderr, "emu launch %lu: grid %u x %u x %u, block %u\n", (unsigned long)n_launches, grid.x, grid.y, grid.z, (unsigned)nt);
    grid_dim = grid;
    block_dim = block;
    nthreads = (int)nt;
    body_fn = &body;
    for (uint32_t bz = 0; bz < grid.z; ++bz)
        for (uint32_t by = 0; by < grid.y; ++by)
            for (uint32_t bx = 0; bx < grid.x; ++bx) {
                for (int i = 0; i < nthreads; ++i) {
                    Thread& t = fibers[i].th;
                    t.flat = (uint32_t)i;
                    t.tid = dim3(i % block.x, (i / block.x) % block.y, i / (block.x * block.y));
                    t.bid = dim3(bx, by, bz);
                }
                ++n_blocks;
                sleep_yields = 0;
                run_block();
                if (abandon) {
                    // fibers of a deadlocked block cannot be unwound; their
                    // stacks are reused by the next block
                    abandon = false;
                    char buf[128];
                    snprintf(buf, sizeof buf, "  (in block %u,%u,%u of a %u-block launch)", bx, by, bz,
                             grid.x * grid.y * grid.z);
                    add_error(buf);
                }
            }
    cur = nullptr;
}

void syncthreads(uintptr_t site) { syncthreads_red(site, -1, 0); }

int syncthreads_red(uintptr_t site, int kind, int v) {
    Fiber* f = running;
    f->site = site;
    f->red_kind = kind;
    f->red_v = v;
    f->st = kAtBarrier;
    to_scheduler();
    return f->red_out;
}

uint64_t wave_op(uintptr_t site, int kind, uint64_t v, int arg) {
    Fiber* f = running;
    f->site = site;
    f->wkind = kind;
    f->wv = v;
    f->warg = arg;
    f->st = kAtWave;
    to_scheduler();
    return f->wout;
}

void maybe_preempt() {
    if (preempt_permille <= 0 || !running) return;
    if ((int)(rng() % 1000) >= preempt_permille) return;
    ++n_preempts;
    to_scheduler();
}

void yield_sleep() {
    if (!running) return;
    if (++sleep_yields == 1000000) add_error("a wait spun 10^6 times inside one workgroup");
    if (sleep_yields > 1000000) return;
    to_scheduler();
}

void note_error(const char* what) { add_error(what); }

}  // namespace emu

// ------------------------------------------------------------ runtime calls
struct emu_stream {
    int dummy;
};
struct emu_event {
    int dummy;
};

hipError_t hipMalloc(void** p, size_t n) {
    *p = malloc(n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    memset(*p, 0xA5, n);  // device memory starts with garbage
    return hipSuccess;
}
hipError_t hipFree(void* p) {
    free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
    *p = malloc(n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
    free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
    if (n) memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
    if (n) memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
    memset(d, v, n);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = new emu_stream();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
    *e = new emu_event();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    *ms = 0.0f;
    return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipPeekAtLastError() { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, int attr, int) {
    *v = attr == hipDeviceAttributeMultiprocessorCount ? 3 : 0;
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "hip error (emulation)"; }

// ------------------------------------------------------------ C entry points
extern "C" {
const char* emu_errors() { return emu::errors.c_str(); }
void emu_clear_errors() { emu::errors.clear(); }
void emu_counts(uint64_t* out) {
    out[0] = emu::n_launches;
    out[1] = emu::n_blocks;
    out[2] = emu::n_barriers;
    out[3] = emu::n_wave_ops;
    out[4] = emu::n_preempts;
}
}
