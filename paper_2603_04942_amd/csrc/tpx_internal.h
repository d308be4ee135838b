// Internal definitions shared by the kernels and the C-ABI layer of libtpx.
// gfx950 (CDNA4) only: 64-lane waves, 160 KB LDS per workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tpx.h"

namespace tpx {

// ---------------------------------------------------------------- format
// TPX3 words (the paper gives no bit layout; this is the library's reading):
//   pixel  0xB | x>>1 (7) | y>>2 (6) | pix (3) | coarse ToA (14) | ToT (10)
//          | fine ToA (4) | spidr (16)
//          x = 2*(x>>1) + (pix>>2), y = 4*(y>>2) + (pix&3)
//          tick = ((spidr<<14 | coarse) << 4) - fine  (mod 2^34)
//   TDC    0x6 | subtype (4) | counter (12) | stamp (35, 3.125 ns) | fine (4)
//          tick = 2 * stamp  (mod 2^36)
// Counter periods: 2^42 and 2^44 chip units of 25/4096 ns (Sec. IV), i.e.
// 2^34 and 2^36 ticks of 1.5625 ns.
constexpr uint64_t kPixPeriod = 1ull << 34;
constexpr uint64_t kTdcPeriod = 1ull << 36;
constexpr uint32_t kHdrPixel = 0xB;
constexpr uint32_t kHdrTdc = 0x6;

enum WordKind : uint32_t { kPixel = 0, kTrigger = 1, kOther = 2, kNone = 3 };

struct Word {
    uint32_t kind, x, y, tot;
    uint64_t raw;
};

__host__ __device__ inline Word decode_word(uint64_t w, uint32_t trig_subtype) {
    Word d;
    d.x = d.y = d.tot = 0;
    d.raw = 0;
    const uint32_t hdr = (uint32_t)(w >> 60);
    if (hdr == kHdrPixel) {
        const uint32_t pix = (uint32_t)(w >> 44) & 7u;
        d.x = (((uint32_t)(w >> 53) & 0x7Fu) << 1) | (pix >> 2);
        d.y = (((uint32_t)(w >> 47) & 0x3Fu) << 2) | (pix & 3u);
        d.tot = (uint32_t)(w >> 20) & 0x3FFu;
        const uint64_t coarse = ((w & 0xFFFFull) << 14) | ((w >> 30) & 0x3FFFull);
        d.raw = ((coarse << 4) - ((w >> 16) & 0xFull)) & (kPixPeriod - 1);
        d.kind = kPixel;
    } else if (hdr == kHdrTdc && ((uint32_t)(w >> 56) & 0xFu) == trig_subtype) {
        d.raw = (((w >> 9) & ((1ull << 35) - 1)) << 1) & (kTdcPeriod - 1);
        d.kind = kTrigger;
    } else {
        d.kind = kOther;
    }
    return d;
}

// Jump of a counter between two consecutive words of one stream (Sec. IV):
// a drop of more than `jump` = the counter wrapped (+1), a rise of more than
// `jump` = a late reporter from before the wrap (-1).
__host__ __device__ inline int jump_of(uint64_t prev, uint64_t cur, uint64_t jump) {
    const int64_t d = (int64_t)cur - (int64_t)prev;
    return d < -(int64_t)jump ? 1 : (d > (int64_t)jump ? -1 : 0);
}

// Summary of a contiguous run of one stream's words, combinable in order.
struct RunSum {
    uint64_t first, last;
    int64_t sum;     // sum of jumps between consecutive words inside the run
    uint64_t count;  // words in the run
};

__host__ __device__ inline RunSum run_empty() { return RunSum{0, 0, 0, 0}; }

__host__ __device__ inline RunSum run_combine(const RunSum& a, const RunSum& b, uint64_t jump) {
    if (a.count == 0) return b;
    if (b.count == 0) return a;
    RunSum r;
    r.first = a.first;
    r.last = b.last;
    r.sum = a.sum + b.sum + jump_of(a.last, b.first, jump);
    r.count = a.count + b.count;
    return r;
}

// ---------------------------------------------------------------- events
// Packed event used between kernels: t (30) | tot (10) | y (8) | x (8).
// t is the time of flight in ticks (stream path) and is limited to 2^30-1.
__host__ __device__ inline uint64_t pack_event(uint32_t x, uint32_t y, uint32_t tot, uint32_t t) {
    return (uint64_t)t | ((uint64_t)tot << 30) | ((uint64_t)y << 40) | ((uint64_t)x << 48);
}
__host__ __device__ inline uint32_t ev_t(uint64_t p) { return (uint32_t)(p & 0x3FFFFFFFull); }
__host__ __device__ inline uint32_t ev_tot(uint64_t p) { return (uint32_t)(p >> 30) & 0x3FFu; }
__host__ __device__ inline uint32_t ev_y(uint64_t p) { return (uint32_t)(p >> 40) & 0xFFu; }
__host__ __device__ inline uint32_t ev_x(uint64_t p) { return (uint32_t)(p >> 48) & 0xFFu; }

// ---------------------------------------------------------------- tiles
constexpr int kTileThreads = 256;
constexpr int kTileItems = 16;
constexpr int kTilePkts = kTileThreads * kTileItems;  // 4096 words = 32 KB
constexpr int kTrigSlice = 512;                        // triggers staged in LDS

// Fold of a run of tiles: pixel and trigger counter runs, trigger words.
struct TileAcc {
    RunSum pix, tdc;
    uint64_t ntrig;
};

__host__ __device__ inline TileAcc acc_empty() { return TileAcc{run_empty(), run_empty(), 0}; }

__host__ __device__ inline TileAcc acc_combine(const TileAcc& a, const TileAcc& b, uint64_t jump) {
    return TileAcc{run_combine(a.pix, b.pix, jump), run_combine(a.tdc, b.tdc, jump),
                   a.ntrig + b.ntrig};
}

struct TileEntry {     // state in force at the start of a tile
    RunSum pix, tdc;   // everything before the tile, folded
    int64_t pix_epoch, tdc_epoch;
    uint64_t trig_off; // triggers before the tile (within this call)
};

// Device-side results and counters of one call; read back with one copy.
struct DevResults {
    unsigned long long err;          // bit mask of kErr*
    unsigned long long n_pixels, n_tdc, n_other, n_pre_trigger, n_tof_cut,
        n_late_drop, n_pix_wraps, n_pix_backjumps, n_tdc_wraps, n_tdc_backjumps;
    unsigned long long n_kept;        // kept events written by this call
    unsigned long long n_trig;        // triggers decoded by this call
    unsigned long long n_hits;        // hits produced
    unsigned long long n_close_ev;    // events of closed shots (stream)
    unsigned long long n_close_grp;   // closed shot groups (stream)
    unsigned long long n_groups;      // shot groups in the event array
    unsigned long long unsorted;      // kept events not in shot order
    unsigned long long max_t_plus1;   // largest unwrapped pixel time + 1 (0 = none)
    unsigned long long seg_ticket, tile_ticket, aux_ticket;
    long long pix_epoch_end, tdc_epoch_end;
    unsigned long long pix_last_end, tdc_last_end, pix_has_end, tdc_has_end;
    unsigned long long big_segments;  // segments clustered in global memory
    unsigned long long max_key;       // largest shot value seen by an event-mode check
    unsigned long long n_in;          // events handed to the cluster kernel (event mode)
    unsigned long long n_close_list;  // closed groups in a sorted group list (fallback)
    unsigned long long carry_last;    // table index of the last carried event + 1 (0 = none)
    unsigned long long n_seg;         // cluster segments of this call
};

enum : unsigned long long {
    kErrStream = 1ull,        // triggers decrease or a wrap count < 0
    kErrInput = 2ull,         // malformed values in an input buffer
    kErrSpin = 4ull,          // a look-back wait exceeded its bound
    kErrCapacity = 8ull,      // an internal buffer was too small
    kErrInternal = 16ull,
    kErrLoopFind = 32ull,     // a union-find walk exceeded the segment size
    kErrLoopUnite = 64ull,    // a union retried more often than possible
    kErrLoopChain = 128ull,   // an image-slot chain was longer than the segment
};

// ---------------------------------------------------------------- look-back
// One 64-bit status word per tile/segment: flag in bits 62-63, value below.
constexpr uint64_t kLbAggregate = 1ull << 62;
constexpr uint64_t kLbInclusive = 2ull << 62;
constexpr uint64_t kLbValueMask = (1ull << 62) - 1;
constexpr uint64_t kLbSpinLimit = 1ull << 26;

__device__ inline void lb_publish(uint64_t* status, uint64_t idx, uint64_t flag, uint64_t v) {
    __hip_atomic_store(status + idx, flag | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Look-back value combiners: plain sums, and for tiles a kept-event count in
// bits 0-30 with the largest kept shot + 1 in bits 31-61.
struct LbSum {
    __device__ static uint64_t op(uint64_t a, uint64_t b) { return a + b; }
};
struct LbCountMax {
    static constexpr uint64_t kLow = (1ull << 31) - 1;
    __device__ static uint64_t op(uint64_t a, uint64_t b) {
        const uint64_t ha = a >> 31, hb = b >> 31;
        return ((a & kLow) + (b & kLow)) | ((ha > hb ? ha : hb) << 31);
    }
};

// Exclusive prefix of the values of items 0..idx-1, called by all 64 lanes of
// one wave: each round reads the status words of the 64 nearest predecessors
// at once and stops at the nearest inclusive one.  A round in which a word
// needed so far is still unpublished is repeated (bounded; kErrSpin).
template <class Op>
__device__ inline uint64_t lb_lookback_wave(uint64_t* status, uint64_t idx, unsigned long long* err) {
    const int l = (int)__lane_id();
    uint64_t acc = 0;
    int64_t base = (int64_t)idx - 1;
    uint64_t spins = 0;
    while (base >= 0) {
        const int64_t j = base - l;
        const uint64_t s = j >= 0 ? __hip_atomic_load(status + j, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT)
                                  : kLbInclusive;  // nothing before item 0
        const uint64_t f = s & ~kLbValueMask;
        const uint64_t incl = __ballot(f == kLbInclusive);
        const uint64_t none = __ballot(f == 0);
        const int fi = incl ? __ffsll((unsigned long long)incl) - 1 : 64;
        const uint64_t need = fi >= 63 ? ~0ull : ((2ull << fi) - 1);
        if (none & need) {
            if (++spins > kLbSpinLimit) {
                if (l == 0) atomicOr(err, (unsigned long long)kErrSpin);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint64_t v = l <= fi ? (s & kLbValueMask) : 0;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) v = Op::op(v, (uint64_t)__shfl_xor(v, d, 64));
        acc = Op::op(acc, v);
        if (fi < 64) break;
        base -= 64;
    }
    return acc;
}

// ---------------------------------------------------------------- waves
__device__ inline uint32_t lane() { return __lane_id(); }

__device__ inline uint64_t lanemask_lt() {
    const uint32_t l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Exclusive prefix sum of a 0/1 flag over a workgroup of NT threads, in
// thread order.  `tmp` holds NT/64 + 1 words of LDS.  Returns the prefix and
// stores the workgroup total in *total.
template <int NT>
__device__ inline uint32_t wg_flag_scan(bool flag, uint32_t* tmp, uint32_t* total) {
    constexpr int NW = NT / 64;
    const uint64_t b = __ballot(flag);
    const uint32_t in_wave = (uint32_t)__popcll(b & lanemask_lt());
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) tmp[w] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const uint32_t c = tmp[k];
        before += (k < w) ? c : 0u;
        all += c;
    }
    __syncthreads();
    *total = all;
    return before + in_wave;
}

// Exclusive prefix sum of a small count over a workgroup, in thread order.
template <int NT>
__device__ inline uint32_t wg_count_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
    constexpr int NW = NT / 64;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d, 64);
        if ((int)__lane_id() >= d) inc += o;
    }
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 63) tmp[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const uint32_t c = tmp[k];
        before += (k < w) ? c : 0u;
        all += c;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

}  // namespace tpx
