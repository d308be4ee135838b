// Device code of the decode, unwrap and shot-assignment passes (tile
// summary, tile entry and trigger unwrap, assignment and placement bodies),
// shared by their kernels (tpx_decode.hip) and the persistent chunk kernel.
#pragma once

#include "tpx_kernels.h"

namespace tpx {


// Packets of one assignment tile are staged through LDS so that each thread
// can walk its consecutive words (coalesced loads; measured faster here than
// each thread reading its own 128 bytes): padded by one word per 16 to
// spread LDS banks.  The same buffer later stages the tile's kept events in
// output order.
__device__ inline int tile_slot(int i) { return i + (i >> 4); }
constexpr int kTileLds = kTilePkts + kTilePkts / 16;
constexpr int kWaves = kTileThreads / 64;
constexpr uint64_t kTrigMargin = 64;   // triggers staged before / after a tile's own
constexpr int kScanTiles = 1024;       // tiles per block of the first scan level

// kItems consecutive words from g0 straight into registers (one thread's
// run of the tile): 16-byte loads when the words are 16-byte aligned (pk is,
// and g0 is a multiple of 8), else 8-byte loads; words at or beyond n read
// as 0.
template <int kItems>
__device__ inline void load_run(const uint64_t* __restrict__ pk, uint64_t g0, uint64_t n,
                                uint64_t (&w)[kItems]) {
    static_assert(kItems % 2 == 0, "pairs of words");
    if (g0 + kItems <= n && (reinterpret_cast<uintptr_t>(pk) & 15u) == 0) {
        const uint4* p = reinterpret_cast<const uint4*>(pk + g0);
#pragma unroll
        for (int k = 0; k < kItems / 2; ++k) {
            const uint4 v = p[k];
            w[2 * k] = (uint64_t)v.x | ((uint64_t)v.y << 32);
            w[2 * k + 1] = (uint64_t)v.z | ((uint64_t)v.w << 32);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) w[k] = g0 + k < n ? __builtin_nontemporal_load(pk + g0 + k) : 0ull;
    }
}

// ------------------------------------------------------------- in-order folds
__device__ inline RunSum run_push(RunSum r, uint64_t raw, uint64_t jump) {
    if (r.count) r.sum += jump_of(r.last, raw, jump); else r.first = raw;
    r.last = raw;
    ++r.count;
    return r;
}

// Cross-lane moves of the data-parallel primitives (DPP) of GFX9: VALU
// operand modifiers, no LDS round trip.  Controls: row_shr:n (from lane
// l - n of the same 16-lane row), row_bcast:15 (lane 15 of the row before),
// row_bcast:31 (lane 31), wave_shr:1 (lane l - 1).
constexpr int kDppRowShr = 0x110, kDppWaveShr1 = 0x138, kDppBcast15 = 0x142,
              kDppBcast31 = 0x143;

// v of the source lane, or `fill` for a lane with no source or outside the
// row mask
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_move(uint32_t v, uint32_t fill) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, kCtrl, kRowMask, 0xf, false);
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint64_t dpp_move(uint64_t v, uint64_t fill) {
    return ((uint64_t)dpp_move<kCtrl, kRowMask>((uint32_t)(v >> 32), (uint32_t)(fill >> 32)) << 32) |
           dpp_move<kCtrl, kRowMask>((uint32_t)v, (uint32_t)fill);
}
// A run moved across lanes (the fill is the empty run); count and sum travel
// as 32 bits (within one wave there are at most 64 x 16 words, so both fit).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ RunSum dpp_move(const RunSum& v, const RunSum&) {
    RunSum o;
    o.first = dpp_move<kCtrl, kRowMask>(v.first, 0ull);
    o.last = dpp_move<kCtrl, kRowMask>(v.last, 0ull);
    o.sum = (int64_t)(int32_t)dpp_move<kCtrl, kRowMask>((uint32_t)v.sum, 0u);
    o.count = dpp_move<kCtrl, kRowMask>((uint32_t)v.count, 0u);
    return o;
}

// Inclusive in-order scan over the lanes of a wave; op(earlier, later), fill
// its identity: within each 16-lane row by shifts of 1, 2, 4 and 8 lanes,
// then rows 1 and 3 take the end of rows 0 and 2, then rows 2 and 3 take the
// end of row 1 (the earlier part is always the left operand, so the order is
// kept).  Every lane must be active; lane 63 ends with the whole wave.
template <class T, class F>
__device__ __forceinline__ T wave_inscan(T v, const T& fill, F op) {
    v = op(dpp_move<kDppRowShr + 1, 0xf>(v, fill), v);
    v = op(dpp_move<kDppRowShr + 2, 0xf>(v, fill), v);
    v = op(dpp_move<kDppRowShr + 4, 0xf>(v, fill), v);
    v = op(dpp_move<kDppRowShr + 8, 0xf>(v, fill), v);
    v = op(dpp_move<kDppBcast15, 0xa>(v, fill), v);
    v = op(dpp_move<kDppBcast31, 0xc>(v, fill), v);
    return v;
}

__device__ inline RunSum wave_run_inscan(RunSum v, uint64_t jump) {
    return wave_inscan(v, run_empty(),
                       [jump](const RunSum& a, const RunSum& b) { return run_combine(a, b, jump); });
}

// Tile and block summaries moved across lanes with every field at full
// width (their counts are not bounded by one wave's words); the fill is the
// empty summary.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ TileAcc dpp_move(const TileAcc& v, const TileAcc&) {
    auto run = [](const RunSum& r) {
        RunSum o;
        o.first = dpp_move<kCtrl, kRowMask>(r.first, (uint64_t)0);
        o.last = dpp_move<kCtrl, kRowMask>(r.last, (uint64_t)0);
        o.sum = (int64_t)dpp_move<kCtrl, kRowMask>((uint64_t)r.sum, (uint64_t)0);
        o.count = dpp_move<kCtrl, kRowMask>(r.count, (uint64_t)0);
        return o;
    };
    return TileAcc{run(v.pix), run(v.tdc), dpp_move<kCtrl, kRowMask>(v.ntrig, (uint64_t)0)};
}

__device__ inline TileAcc wave_acc_inscan(TileAcc v, uint64_t jump) {
    return wave_inscan(v, acc_empty(),
                       [jump](const TileAcc& a, const TileAcc& b) { return acc_combine(a, b, jump); });
}

// exclusive form of an inclusive scan: lane 0 gets the empty summary
__device__ inline TileAcc wave_acc_shift1(const TileAcc& inc) {
    return dpp_move<kDppWaveShr1, 0xf>(inc, acc_empty());
}

// Exclusive in-order fold of one RunSum per thread over a workgroup of NW
// waves; *all gets the fold of every thread.  wbuf holds one entry per wave.
template <int NW = kWaves>
__device__ inline RunSum wg_run_exscan(RunSum v, RunSum* wbuf, uint64_t jump, RunSum* all) {
    const RunSum inc = wave_run_inscan(v, jump);
    const RunSum ex = dpp_move<kDppWaveShr1, 0xf>(inc, run_empty());  // lane 0: empty
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 63) wbuf[w] = inc;
    __syncthreads();
    RunSum pre = run_empty(), tot = run_empty();
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const RunSum c = wbuf[k];
        if (k < w) pre = run_combine(pre, c, jump);
        tot = run_combine(tot, c, jump);
    }
    __syncthreads();
    *all = tot;
    return run_combine(pre, ex, jump);
}

// Exclusive in-order fold of one TileAcc per thread over 1024 threads.
__device__ inline TileAcc wg1024_acc_exscan(TileAcc v, TileAcc* wbuf, uint64_t jump,
                                            TileAcc* all) {
    const TileAcc inc = wave_acc_inscan(v, jump);
    const TileAcc ex = wave_acc_shift1(inc);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 63) wbuf[w] = inc;
    __syncthreads();
    TileAcc pre = acc_empty(), tot = acc_empty();
    for (int k = 0; k < 16; ++k) {
        const TileAcc c = wbuf[k];
        if (k < w) pre = acc_combine(pre, c, jump);
        tot = acc_combine(tot, c, jump);
    }
    __syncthreads();
    *all = tot;
    return acc_combine(pre, ex, jump);
}

// ------------------------------------------------------------------ summary
// 512 threads of 8 consecutive words per tile, read straight into registers.
constexpr int kSumThreads = 512;
constexpr int kSumItems = kTilePkts / kSumThreads;
constexpr int kSumWaves = kSumThreads / 64;

__device__ __forceinline__ void tile_summary_body(const uint64_t* __restrict__ pk, uint64_t n,
                                                  uint32_t sub, uint64_t jump, TileAcc* sums,
                                                  uint64_t* tdc_slot, uint64_t tile, RunSum* wbuf,
                                                  uint32_t* tmp) {
    const uint64_t base = tile * kTilePkts;
    const uint64_t g0 = base + (uint64_t)threadIdx.x * kSumItems;
    uint64_t wd[kSumItems];
    load_run<kSumItems>(pk, g0, n, wd);
    RunSum P = run_empty(), T = run_empty();
#pragma unroll
    for (int j = 0; j < kSumItems; ++j) {
        if (g0 + j < n) {
            const Word d = decode_word(wd[j], sub);
            if (d.kind == kPixel) P = run_push(P, d.raw, jump);
            else if (d.kind == kTrigger) T = run_push(T, d.raw, jump);
        }
    }
    uint32_t ntot;
    const uint32_t nt = (uint32_t)T.count;
    const uint32_t pos = wg_count_scan<kSumThreads>(nt, tmp, &ntot);
    if (nt) {
        uint32_t q = 0;
#pragma unroll
        for (int j = 0; j < kSumItems; ++j) {
            if (g0 + j < n) {
                const Word d = decode_word(wd[j], sub);
                if (d.kind == kTrigger) tdc_slot[base + pos + q++] = d.raw;
            }
        }
    }
    RunSum ap, at;
    wg_run_exscan<kSumWaves>(P, wbuf, jump, &ap);
    wg_run_exscan<kSumWaves>(T, wbuf, jump, &at);
    if (threadIdx.x == 0) sums[tile] = TileAcc{ap, at, ntot};
}

// One tile (one thread): its entry state from `pre` (the fold of the state
// in force at the call's start and every earlier tile; init_ntrig = the
// trigger count of that initial state), then its trigger words in order.
__device__ __forceinline__ void unwrap_tile(const TileAcc& pre, uint64_t init_ntrig, uint64_t tile,
                                   const TileAcc* __restrict__ sums,
                                   const uint64_t* __restrict__ tdc_slot, int64_t pe0, int64_t te0,
                                   uint64_t jump, TileEntry* entries, uint64_t* tab,
                                   DevResults* res) {
    TileEntry e;
    e.pix = pre.pix;
    e.tdc = pre.tdc;
    e.pix_epoch = pe0 + pre.pix.sum;
    e.tdc_epoch = te0 + pre.tdc.sum;
    e.trig_off = pre.ntrig - init_ntrig;
    entries[tile] = e;
    const uint32_t c = (uint32_t)sums[tile].ntrig;
    if (c == 0) return;
    bool has = e.tdc.count > 0;
    uint64_t last = e.tdc.last;
    int64_t epoch = e.tdc_epoch;
    bool has_prev_t = has && epoch >= 0;
    uint64_t prev_t = has ? last + (uint64_t)epoch * kTdcPeriod : 0;
    unsigned long long fwd = 0, back = 0, err = 0;
    for (uint32_t q = 0; q < c; ++q) {
        const uint64_t raw = tdc_slot[tile * kTilePkts + q];
        if (has) {
            const int j = jump_of(last, raw, jump);
            epoch += j;
            fwd += j > 0;
            back += j < 0;
        }
        has = true;
        last = raw;
        if (epoch < 0) {
            err |= kErrStream;
            break;
        }
        const uint64_t tt = raw + (uint64_t)epoch * kTdcPeriod;
        if (has_prev_t && tt < prev_t) err |= kErrStream;
        prev_t = tt;
        has_prev_t = true;
        tab[e.trig_off + q] = tt;
    }
    if (fwd) atomicAdd(&res->n_tdc_wraps, fwd);
    if (back) atomicAdd(&res->n_tdc_backjumps, back);
    if (err) atomicOr(&res->err, err);
}

// upper_bound over a sorted array: first index with a[i] > v, in [lo, hi)
template <typename P>
__device__ inline uint64_t upper_bound_u64(P a, uint64_t lo, uint64_t hi, uint64_t v) {
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------- assign
// kStaged (packed output only): tile = workgroup index, no look-back; the
// kept events go to the tile's own staging range and the tile's counts,
// shot range and statistics to per-tile records.
// Packed output (the stream path) reads each thread's words straight into
// registers and writes its kept events from there; the SoA output stages the
// tile through LDS.
constexpr bool kAssignDirect = true;

// LDS of one assignment workgroup of kThreads threads
template <int kThreads, bool kSoA = false>
struct AssignLds {
    static constexpr int kItems = kTilePkts / kThreads;  // consecutive words per thread
    static constexpr int kW = kThreads / 64;
    static constexpr bool kDirect = kAssignDirect && !kSoA;
    uint64_t sp[kDirect ? 2 : kTileLds];
    uint64_t slice[kTrigSlice + 1];
    RunSum wbuf[kW];
    uint32_t w_cnt[kW], w_max[kW], w_min[kW];
    unsigned long long w_stat[kW][8];
    uint64_t bcast[2];
};

template <bool kSoA, bool kStaged, int kThreads>
__device__ __forceinline__ void assign_body(const AssignArgs& a, uint32_t tile_staged,
                                            AssignLds<kThreads, kSoA>& L) {
    using LdsT = AssignLds<kThreads, kSoA>;
    constexpr int kItems = LdsT::kItems, kW = LdsT::kW;
    constexpr bool kDirect = LdsT::kDirect;
    uint64_t* sp = L.sp;
    uint64_t* slice = L.slice;
    uint64_t* bcast = L.bcast;
    constexpr uint32_t kNo = 0xFFFFFFFFu;

    uint32_t tile;
    if constexpr (kStaged) {
        tile = tile_staged;
    } else {
        if (threadIdx.x == 0) bcast[0] = atomicAdd(&a.res->tile_ticket, 1ull);
        __syncthreads();
        tile = __builtin_amdgcn_readfirstlane((uint32_t)bcast[0]);
    }
    const uint64_t base = (uint64_t)tile * kTilePkts;
    uint64_t rw[kDirect ? kItems : 1];
    if constexpr (kDirect) {
        load_run<kItems>(a.pk, base + (uint64_t)threadIdx.x * kItems, a.n, rw);
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int i = k * kThreads + threadIdx.x;
            const uint64_t g = base + (uint64_t)i;
            sp[tile_slot(i)] = g < a.n ? __builtin_nontemporal_load(a.pk + g) : 0ull;
        }
    }
    const TileEntry e = a.entries[tile];
    const uint64_t n_tab = a.n_win + *a.n_trig_dev;
    // slice of the trigger table around this tile's own trigger words
    const uint64_t t0 = a.n_win + e.trig_off;
    const uint64_t s_lo = t0 > kTrigMargin ? t0 - kTrigMargin : 0;
    uint64_t s_hi = min<uint64_t>(n_tab, t0 + a.sums[tile].ntrig + kTrigMargin);
    s_hi = min<uint64_t>(s_hi, s_lo + kTrigSlice);
    const uint32_t len = (uint32_t)(s_hi - s_lo);
    const bool has_above = s_hi < n_tab;  // slice[len] = tab[s_hi]
    for (uint32_t k = threadIdx.x; k < len + (has_above ? 1u : 0u); k += kThreads)
        slice[k] = a.tab[s_lo + k];
    __syncthreads();
    const int nvalid = (int)min<uint64_t>((uint64_t)kTilePkts, a.n - base);

    // every word decoded once: a pixel as raw tick | x << 34 | y << 42 |
    // ToT << 50, anything else as a marker; the thread's run of pixel counter
    // values is folded across the workgroup
    constexpr uint64_t kNotPixel = 1ull << 63, kOtherWord = 1ull << 62;
    uint64_t tv[kItems];
    RunSum P = run_empty();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int i = threadIdx.x * kItems + j;
        tv[j] = kNotPixel;
        if (i < nvalid) {
            const Word d = decode_word(kDirect ? rw[kDirect ? j : 0] : sp[tile_slot(i)], a.sub);
            if (d.kind == kPixel) {
                tv[j] = d.raw | ((uint64_t)d.x << 34) | ((uint64_t)d.y << 42) | ((uint64_t)d.tot << 50);
                P = run_push(P, d.raw, a.jump);
            } else if (d.kind == kOther) {
                tv[j] = kNotPixel | kOtherWord;
            }
        }
    }
    RunSum all;
    const RunSum pre = run_combine(e.pix, wg_run_exscan<kW>(P, L.wbuf, a.jump, &all), a.jump);

    // unwrap, then the shot of each pixel (latest trigger at or before it),
    // ToF cut, keep; tv[j] becomes the kept event (or ~0)
    bool has = pre.count > 0;
    uint64_t last = pre.last;
    int64_t epoch = e.pix_epoch + (pre.sum - e.pix.sum);
    uint64_t tmax1 = 0;
    uint32_t fwd = 0, back = 0, npix = 0, nother = 0;
    unsigned long long err = 0;
    uint32_t sv[kItems];
    uint32_t nkeep = 0, npre = 0, ncut = 0, nlate = 0;
    uint32_t first_s = kNo, last_s = 0;
    bool sorted = true;
    // the slice interval [h_lo, h_hi) of the last search, in registers:
    // consecutive pixels mostly fall in the same shot, so most need no LDS
    // read (h_lo = 0 stands for "no entry before", h_hi = ~0 for "no entry
    // after" within the slice)
    uint32_t hint = 0;
    uint64_t h_lo = 0, h_hi = len ? slice[0] : ~0ull;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        sv[j] = kNo;
        const uint64_t dv = tv[j];
        tv[j] = ~0ull;
        if (dv & kNotPixel) {
            nother += (dv & kOtherWord) ? 1u : 0u;
            continue;
        }
        const uint64_t raw = dv & (kPixPeriod - 1);
        if (has) {
            const int jj = jump_of(last, raw, a.jump);
            epoch += jj;
            fwd += jj > 0;
            back += jj < 0;
        }
        has = true;
        last = raw;
        ++npix;
        if (epoch < 0) {
            err |= kErrStream;
            continue;
        }
        const uint64_t t = raw + (uint64_t)epoch * kPixPeriod;
        tmax1 = max(tmax1, t + 1);
        uint64_t ub, trig;
        const bool below = s_lo > 0 && t < slice[0];
        const bool above = has_above && t >= slice[len];
        if (!below && !above) {
            // entries before the slice are <= t, entries after it are > t
            if (!(h_lo <= t && t < h_hi)) {
                hint = (uint32_t)upper_bound_u64(slice, 0, len, t);
                h_lo = hint ? slice[hint - 1] : 0;
                h_hi = hint < len ? slice[hint] : ~0ull;
            }
            ub = s_lo + hint;
            trig = h_lo;
        } else {
            ub = upper_bound_u64(a.tab, 0, n_tab, t);
            trig = ub ? a.tab[ub - 1] : 0;
        }
        if (ub == 0) {
            if (a.tab_has_before) ++nlate; else ++npre;
        } else {
            const uint64_t s = ub - 1;
            const uint64_t tof = t - trig;
            if (tof > a.tof_max) {
                ++ncut;
            } else if (s < a.first_open) {
                ++nlate;
            } else {
                sv[j] = (uint32_t)s;
                ++nkeep;
                if (first_s == kNo) first_s = (uint32_t)s;
                if ((uint32_t)s < last_s) sorted = false;
                last_s = (uint32_t)s;
                if constexpr (kSoA) {
                    tv[j] = t;
                } else {
                    tv[j] = pack_event((uint32_t)(dv >> 34) & 255u, (uint32_t)(dv >> 42) & 255u,
                                       (uint32_t)(dv >> 50) & 1023u, (uint32_t)tof);
                }
            }
        }
    }

    // workgroup: kept-event prefix, running max of kept shots (order check),
    // smallest kept shot, statistics
    const int w = threadIdx.x >> 6;
    const uint32_t m1 = nkeep ? last_s + 1 : 0;
    // (inclusive scans over the wave; lane 63 holds the wave's totals)
    auto add32 = [](uint32_t x, uint32_t y) { return x + y; };
    auto max32 = [](uint32_t x, uint32_t y) { return max(x, y); };
    auto min32 = [](uint32_t x, uint32_t y) { return min(x, y); };
    auto add64 = [](uint64_t x, uint64_t y) { return x + y; };
    auto max64 = [](uint64_t x, uint64_t y) { return max(x, y); };
    const uint32_t cinc = wave_inscan(nkeep, 0u, add32), minc = wave_inscan(m1, 0u, max32);
    const uint32_t fmin = wave_inscan(nkeep ? first_s : kNo, kNo, min32);
    // the seven per-thread counts (each <= 16) in 16-bit fields of two words
    // (a wave's sums stay below 2^16 in every field)
    const uint64_t st0 = wave_inscan((uint64_t)npix | ((uint64_t)nother << 16) |
                                         ((uint64_t)npre << 32) | ((uint64_t)ncut << 48),
                                     (uint64_t)0, add64);
    const uint64_t st1 = wave_inscan((uint64_t)nlate | ((uint64_t)fwd << 16) | ((uint64_t)back << 32),
                                     (uint64_t)0, add64);
    const uint32_t stat[7] = {(uint32_t)(st0 & 0xFFFF), (uint32_t)((st0 >> 16) & 0xFFFF),
                              (uint32_t)((st0 >> 32) & 0xFFFF), (uint32_t)(st0 >> 48),
                              (uint32_t)(st1 & 0xFFFF), (uint32_t)((st1 >> 16) & 0xFFFF),
                              (uint32_t)((st1 >> 32) & 0xFFFF)};
    const uint64_t tm = wave_inscan(tmax1, (uint64_t)0, max64);
    if (__lane_id() == 63) {
        L.w_cnt[w] = cinc;
        L.w_max[w] = minc;
        L.w_min[w] = fmin;
#pragma unroll
        for (int k = 0; k < 7; ++k) L.w_stat[w][k] = stat[k];
        L.w_stat[w][7] = tm;
    }
    const uint32_t mex_w = dpp_move<kDppWaveShr1, 0xf>(minc, 0u);  // lane 0: 0
    __syncthreads();
    uint32_t tpre = cinc - nkeep, mex = mex_w, tile_keep = 0, tile_max1 = 0, tile_min = kNo;
#pragma unroll
    for (int k = 0; k < kW; ++k) {
        if (k < w) {
            tpre += L.w_cnt[k];
            mex = max(mex, L.w_max[k]);
        }
        tile_keep += L.w_cnt[k];
        tile_max1 = max(tile_max1, L.w_max[k]);
        tile_min = min(tile_min, L.w_min[k]);
    }
    const bool bad = !sorted || (nkeep && first_s + 1 < mex);
    const bool tile_bad = __syncthreads_or(bad) != 0;

    if constexpr (kStaged) {
        // per-tile records instead of a look-back
        if (threadIdx.x == 0) {
            a.tile_cnt[tile] = tile_keep;
            a.tile_lo[tile] = tile_keep ? tile_min : kNo;
            a.tile_hi[tile] = tile_max1;
            if (tile_bad) atomicOr(&a.res->unsorted, 1ull);
            unsigned long long* st = a.tile_stat + 8ull * tile;
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                unsigned long long v = 0;
                for (int q = 0; q < kW; ++q) v += L.w_stat[q][k];
                st[k] = v;
            }
            unsigned long long mx = 0;
            for (int q = 0; q < kW; ++q) mx = max(mx, L.w_stat[q][7]);
            st[7] = mx;
            bcast[1] = 0;
        }
    } else if (w == 0) {
        // look-back over tiles: kept events and largest kept shot before this tile
        const uint64_t mine = (uint64_t)tile_keep | ((uint64_t)tile_max1 << 31);
        uint64_t prefix;
        if (tile == 0) {
            prefix = a.carry_last1 << 31;
        } else {
            if (__lane_id() == 0) lb_publish(a.lb_status, tile, kLbAggregate, mine);
            prefix = lb_lookback_wave<LbCountMax>(a.lb_status, tile, &a.res->err);
        }
        if (__lane_id() == 0) {
            lb_publish(a.lb_status, tile, kLbInclusive, LbCountMax::op(prefix, mine));
            bcast[1] = prefix;
            const uint64_t prev_max1 = prefix >> 31;
            if (tile_bad || (tile_keep && prev_max1 > (uint64_t)tile_min + 1))
                atomicOr(&a.res->unsorted, 1ull);
            unsigned long long* dst[7] = {&a.res->n_pixels, &a.res->n_other, &a.res->n_pre_trigger,
                                          &a.res->n_tof_cut, &a.res->n_late_drop,
                                          &a.res->n_pix_wraps, &a.res->n_pix_backjumps};
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                unsigned long long v = 0;
                for (int q = 0; q < kW; ++q) v += L.w_stat[q][k];
                if (v) atomicAdd(dst[k], v);
            }
            unsigned long long mx = 0;
            for (int q = 0; q < kW; ++q) mx = max(mx, L.w_stat[q][7]);
            if (mx) atomicMax(&a.res->max_t_plus1, mx);
            if (tile_keep) atomicAdd(&a.res->n_kept, (unsigned long long)tile_keep);
        }
    }
    if (err) atomicOr(&a.res->err, err);
    __syncthreads();
    const uint64_t pcount = bcast[1] & LbCountMax::kLow;
    const uint64_t out0 = kStaged ? (uint64_t)tile * kTilePkts : a.ev_off + pcount;

    if constexpr (kSoA) {
        uint64_t o = out0 + tpre;
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            if (sv[j] != kNo) {
                if (o < a.ev_cap) {
                    const Word d = decode_word(sp[tile_slot(threadIdx.x * kItems + j)], a.sub);
                    a.soa.x[o] = (uint16_t)d.x;
                    a.soa.y[o] = (uint16_t)d.y;
                    a.soa.tot[o] = (uint16_t)d.tot;
                    a.soa.shot[o] = (uint32_t)(a.shot_base + sv[j]);
                    a.soa.toa[o] = tv[j];
                }
                ++o;
            }
        }
    } else {
        if constexpr (kDirect) {
            // kept events (and shots) from registers, each thread's in order
            uint64_t o = out0 + tpre;
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                if (sv[j] != kNo) {
                    if (o < a.ev_cap) {
                        a.ev[o] = tv[j];
                        if (a.shot_out) a.shot_out[o] = sv[j];
                    }
                    ++o;
                }
            }
        } else {
            // kept events staged in LDS in output order, then written contiguously
            {
                uint32_t q = tpre;
#pragma unroll
                for (int j = 0; j < kItems; ++j)
                    if (sv[j] != kNo) sp[tile_slot(q++)] = tv[j];
            }
            __syncthreads();
            for (uint32_t k = threadIdx.x; k < tile_keep; k += kThreads)
                if (out0 + k < a.ev_cap) a.ev[out0 + k] = sp[tile_slot(k)];
            if (a.shot_out) {
                __syncthreads();
                uint32_t q = tpre;
#pragma unroll
                for (int j = 0; j < kItems; ++j)
                    if (sv[j] != kNo) sp[tile_slot(q++)] = sv[j];
                __syncthreads();
                for (uint32_t k = threadIdx.x; k < tile_keep; k += kThreads)
                    if (out0 + k < a.ev_cap) a.shot_out[out0 + k] = (uint32_t)sp[tile_slot(k)];
            }
        }
        // events per shot from run boundaries: a run of shot s over positions
        // [p, p') adds p' - p to its count.  Exact when the kept events are in
        // shot order (otherwise the caller takes the sorting path).
        if (a.shot_cnt && nkeep) {
            uint32_t prev = mex;  // previous kept shot in the tile + 1, 0 = none
            uint32_t p = (uint32_t)(pcount + tpre);
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                const uint32_t s = sv[j];
                if (s != kNo) {
                    if (prev == 0) {
                        atomicAdd(&a.shot_cnt[s], 0u - p);
                    } else if (prev - 1 != s) {
                        atomicAdd(&a.shot_cnt[prev - 1], p);
                        atomicAdd(&a.shot_cnt[s], 0u - p);
                    }
                    prev = s + 1;
                    ++p;
                }
            }
            if (tpre + nkeep == tile_keep) atomicAdd(&a.shot_cnt[prev - 1], p);
        }
    }
}

// Staged kept events of tile t to their place; the shot order across tiles
// (a tile's smallest kept shot below the largest of the nearest earlier tile
// with kept events, or of the carried events); the call's kept-event count.
constexpr int kPlaceThreads = 256;
__device__ __forceinline__ void place_tile(const AssignArgs& a, const uint32_t* tile_off,
                                           uint64_t* ev_out, uint64_t ev_off, uint64_t ev_cap,
                                           uint32_t* shot_final, uint64_t ntiles, uint64_t t,
                                           uint32_t nthreads) {
    if (t == 0 && threadIdx.x == 0) a.res->n_kept = tile_off[ntiles];
    const uint32_t cnt = a.tile_cnt[t];
    const uint64_t src = t * kTilePkts, dst = ev_off + tile_off[t];
    for (uint32_t k = threadIdx.x; k < cnt; k += nthreads) {
        if (dst + k >= ev_cap) break;
        ev_out[dst + k] = a.ev[src + k];
        if (shot_final) shot_final[dst + k] = a.shot_out[src + k];
    }
    if (threadIdx.x == 0 && cnt) {
        // the nearest earlier tile with kept events holds kept position
        // tile_off[t] - 1: the last t' < t with tile_off[t'] <= it
        uint64_t prev_max1 = a.carry_last1;
        const uint32_t before = tile_off[t];
        if (before > 0) {
            uint64_t lo = 0, hi = t;  // tile_off[lo] <= before - 1 < tile_off[hi]
            while (hi - lo > 1) {
                const uint64_t mid = (lo + hi) >> 1;
                if (tile_off[mid] <= before - 1) lo = mid; else hi = mid;
            }
            prev_max1 = a.tile_hi[lo];
        }
        if (prev_max1 > (uint64_t)a.tile_lo[t] + 1) atomicOr(&a.res->unsorted, 1ull);
    }
}

}  // namespace tpx
