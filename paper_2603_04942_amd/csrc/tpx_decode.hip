// Decode, unwrap and shot assignment (Sec. III; Sec. IV, ToA Unwrapping and
// Eliminating Background Counts) as passes over 4096-word tiles:
//   k_tile_summary  per tile: folded pixel / trigger counter runs and the
//                   trigger words in stream order (one read of the packets);
//   k_tile_scan1/2  fold the tile summaries into the state in force at the
//                   start of every tile (blocks of 1024 tiles, then blocks);
//   k_trig_unwrap   one thread per tile: its entry state, and its trigger
//                   words unwrapped into the trigger table;
//   k_assign        second read of the packets: unwraps each pixel, finds its
//                   shot (latest trigger at or before it) in a slice of the
//                   trigger table staged in LDS, applies the ToF cut and
//                   writes the kept events in stream order (stable compaction
//                   with a decoupled look-back over tiles that also checks
//                   that kept events are in shot order).
#include "tpx_kernels.h"

namespace tpx {

// Packets of one tile staged through LDS so that each thread can walk 16
// consecutive words (coalesced loads; measured faster here than each thread
// reading its own 128 bytes): padded by one word per 16 to spread LDS banks.
// The same buffer later stages the tile's kept events in output order.
__device__ inline int tile_slot(int i) { return i + (i >> 4); }
constexpr int kTileLds = kTilePkts + kTilePkts / 16;
constexpr int kWaves = kTileThreads / 64;
constexpr uint64_t kTrigMargin = 64;   // triggers staged before / after a tile's own
constexpr int kScanTiles = 1024;       // tiles per block of the first scan level

__device__ inline void load_tile(const uint64_t* __restrict__ pk, uint64_t base, uint64_t n,
                                 uint64_t* sp) {
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        const int i = k * kTileThreads + threadIdx.x;
        const uint64_t g = base + (uint64_t)i;
        sp[tile_slot(i)] = g < n ? __builtin_nontemporal_load(pk + g) : 0ull;
    }
}

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

__device__ inline RunSum shfl_up_run(const RunSum& v, int d) {
    RunSum o;
    o.first = __shfl_up(v.first, d, 64);
    o.last = __shfl_up(v.last, d, 64);
    o.sum = __shfl_up(v.sum, d, 64);
    o.count = __shfl_up(v.count, d, 64);
    return o;
}

__device__ inline TileAcc shfl_up_acc(const TileAcc& v, int d) {
    return TileAcc{shfl_up_run(v.pix, d), shfl_up_run(v.tdc, d), __shfl_up(v.ntrig, d, 64)};
}

// Inclusive in-order fold over the lanes of a wave (Kogge-Stone).
__device__ inline RunSum wave_run_inscan(RunSum v, uint64_t jump) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const RunSum o = shfl_up_run(v, d);
        if ((int)__lane_id() >= d) v = run_combine(o, v, jump);
    }
    return v;
}

__device__ inline TileAcc wave_acc_inscan(TileAcc v, uint64_t jump) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const TileAcc o = shfl_up_acc(v, d);
        if ((int)__lane_id() >= d) v = acc_combine(o, v, jump);
    }
    return v;
}

// Exclusive in-order fold of one RunSum per thread over a workgroup of NW
// waves; *all gets the fold of every thread.  wbuf holds one entry per wave.
template <int NW = kWaves>
__device__ inline RunSum wg_run_exscan(RunSum v, RunSum* wbuf, uint64_t jump, RunSum* all) {
    const RunSum inc = wave_run_inscan(v, jump);
    RunSum ex = shfl_up_run(inc, 1);
    if (__lane_id() == 0) ex = run_empty();
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
    TileAcc ex = shfl_up_acc(inc, 1);
    if (__lane_id() == 0) ex = acc_empty();
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

__global__ __launch_bounds__(kSumThreads) void k_tile_summary(const uint64_t* __restrict__ pk,
                                                             uint64_t n, uint32_t sub,
                                                             uint64_t jump, TileAcc* sums,
                                                             uint64_t* tdc_slot) {
    __shared__ RunSum wbuf[kSumWaves];
    __shared__ uint32_t tmp[kSumWaves + 1];
    const uint64_t tile = blockIdx.x;
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

// -------------------------------------------------------------- tile prefix
// First level: exclusive fold of the tiles inside each block of 1024 tiles
// (partial) and the fold of every block (blk[b]).
__global__ __launch_bounds__(1024) void k_tile_scan1(const TileAcc* __restrict__ sums,
                                                    uint64_t ntiles, uint64_t jump,
                                                    TileAcc* partial, TileAcc* blk) {
    __shared__ TileAcc wbuf[16];
    const uint64_t t = (uint64_t)blockIdx.x * kScanTiles + threadIdx.x;
    const TileAcc v = t < ntiles ? sums[t] : acc_empty();
    TileAcc all;
    const TileAcc ex = wg1024_acc_exscan(v, wbuf, jump, &all);
    if (t < ntiles) partial[t] = ex;
    if (threadIdx.x == 0) blk[blockIdx.x] = all;
}

// Second level (one workgroup): state in force at the start of every block,
// blk[nblk + b], and the state at the end of the call.
__global__ __launch_bounds__(1024) void k_tile_scan2(TileAcc* blk, uint64_t nblk, TileAcc init,
                                                    int64_t pe0, int64_t te0, uint64_t jump,
                                                    DevResults* res) {
    __shared__ TileAcc wbuf[16];
    const uint64_t b = threadIdx.x;
    TileAcc v = b < nblk ? blk[b] : acc_empty();
    if (b == 0) v = acc_combine(init, v, jump);
    TileAcc all;
    TileAcc ex = wg1024_acc_exscan(v, wbuf, jump, &all);
    if (b == 0) ex = init;
    if (b < nblk) blk[nblk + b] = ex;
    if (b == 0) {
        res->pix_epoch_end = pe0 + all.pix.sum;
        res->tdc_epoch_end = te0 + all.tdc.sum;
        res->pix_last_end = all.pix.last;
        res->tdc_last_end = all.tdc.last;
        res->pix_has_end = all.pix.count > 0;
        res->tdc_has_end = all.tdc.count > 0;
        res->n_trig = all.ntrig - init.ntrig;
    }
}

// One thread per tile: its entry state, then its trigger words in order.
__global__ void k_trig_unwrap(const TileAcc* __restrict__ sums, const TileAcc* __restrict__ partial,
                              const TileAcc* __restrict__ blk, const uint64_t* __restrict__ tdc_slot,
                              uint64_t ntiles, uint64_t nblk, int64_t pe0, int64_t te0,
                              uint64_t jump, TileEntry* entries, uint64_t* tab, DevResults* res) {
    const uint64_t tile = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    const TileAcc pre = acc_combine(blk[nblk + tile / kScanTiles], partial[tile], jump);
    TileEntry e;
    e.pix = pre.pix;
    e.tdc = pre.tdc;
    e.pix_epoch = pe0 + pre.pix.sum;
    e.tdc_epoch = te0 + pre.tdc.sum;
    e.trig_off = pre.ntrig - blk[nblk].ntrig;  // init.ntrig is the front of block 0
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
template <bool kSoA, bool kStaged = false>
__global__ __launch_bounds__(kTileThreads) void k_assign(AssignArgs a) {
    __shared__ uint64_t sp[kTileLds];
    __shared__ uint64_t slice[kTrigSlice + 1];
    __shared__ RunSum wbuf[kWaves];
    __shared__ uint32_t w_cnt[kWaves], w_max[kWaves], w_min[kWaves];
    __shared__ unsigned long long w_stat[kWaves][8];
    __shared__ uint64_t bcast[2];
    constexpr uint32_t kNo = 0xFFFFFFFFu;

    uint32_t tile;
    if constexpr (kStaged) {
        tile = blockIdx.x;
    } else {
        if (threadIdx.x == 0) bcast[0] = atomicAdd(&a.res->tile_ticket, 1ull);
        __syncthreads();
        tile = __builtin_amdgcn_readfirstlane((uint32_t)bcast[0]);
    }
    const uint64_t base = (uint64_t)tile * kTilePkts;
    load_tile(a.pk, base, a.n, sp);
    const TileEntry e = a.entries[tile];
    const uint64_t n_tab = a.n_win + *a.n_trig_dev;
    // slice of the trigger table around this tile's own trigger words
    const uint64_t t0 = a.n_win + e.trig_off;
    const uint64_t s_lo = t0 > kTrigMargin ? t0 - kTrigMargin : 0;
    uint64_t s_hi = min<uint64_t>(n_tab, t0 + a.sums[tile].ntrig + kTrigMargin);
    s_hi = min<uint64_t>(s_hi, s_lo + kTrigSlice);
    const uint32_t len = (uint32_t)(s_hi - s_lo);
    const bool has_above = s_hi < n_tab;  // slice[len] = tab[s_hi]
    for (uint32_t k = threadIdx.x; k < len + (has_above ? 1u : 0u); k += kTileThreads)
        slice[k] = a.tab[s_lo + k];
    __syncthreads();
    const int nvalid = (int)min<uint64_t>((uint64_t)kTilePkts, a.n - base);

    // every word decoded once: a pixel as raw tick | x << 34 | y << 42 |
    // ToT << 50, anything else as a marker; the thread's run of pixel counter
    // values is folded across the workgroup
    constexpr uint64_t kNotPixel = 1ull << 63, kOtherWord = 1ull << 62;
    uint64_t tv[kTileItems];
    RunSum P = run_empty();
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
        const int i = threadIdx.x * kTileItems + j;
        tv[j] = kNotPixel;
        if (i < nvalid) {
            const Word d = decode_word(sp[tile_slot(i)], a.sub);
            if (d.kind == kPixel) {
                tv[j] = d.raw | ((uint64_t)d.x << 34) | ((uint64_t)d.y << 42) | ((uint64_t)d.tot << 50);
                P = run_push(P, d.raw, a.jump);
            } else if (d.kind == kOther) {
                tv[j] = kNotPixel | kOtherWord;
            }
        }
    }
    RunSum all;
    const RunSum pre = run_combine(e.pix, wg_run_exscan(P, wbuf, a.jump, &all), a.jump);

    // unwrap, then the shot of each pixel (latest trigger at or before it),
    // ToF cut, keep; tv[j] becomes the kept event (or ~0)
    bool has = pre.count > 0;
    uint64_t last = pre.last;
    int64_t epoch = e.pix_epoch + (pre.sum - e.pix.sum);
    uint64_t tmax1 = 0;
    uint32_t fwd = 0, back = 0, npix = 0, nother = 0;
    unsigned long long err = 0;
    uint32_t sv[kTileItems];
    uint32_t nkeep = 0, npre = 0, ncut = 0, nlate = 0;
    uint32_t first_s = kNo, last_s = 0;
    bool sorted = true;
    uint32_t hint = 0;
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
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
            const bool ok = (hint == 0 || slice[hint - 1] <= t) && (hint == len || t < slice[hint]);
            if (!ok) hint = (uint32_t)upper_bound_u64(slice, 0, len, t);
            ub = s_lo + hint;
            trig = hint ? slice[hint - 1] : 0;
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
    uint32_t cinc = nkeep, minc = m1, fmin = nkeep ? first_s : kNo;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t oc = __shfl_up(cinc, d, 64), om = __shfl_up(minc, d, 64);
        if ((int)__lane_id() >= d) {
            cinc += oc;
            minc = max(minc, om);
        }
        fmin = min(fmin, (uint32_t)__shfl_xor(fmin, d, 64));
    }
    // the seven per-thread counts (each <= 16) in 16-bit fields of two words
    uint64_t st0 = (uint64_t)npix | ((uint64_t)nother << 16) | ((uint64_t)npre << 32) |
                   ((uint64_t)ncut << 48);
    uint64_t st1 = (uint64_t)nlate | ((uint64_t)fwd << 16) | ((uint64_t)back << 32);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        st0 += __shfl_xor(st0, d, 64);
        st1 += __shfl_xor(st1, d, 64);
    }
    const uint32_t stat[7] = {(uint32_t)(st0 & 0xFFFF), (uint32_t)((st0 >> 16) & 0xFFFF),
                              (uint32_t)((st0 >> 32) & 0xFFFF), (uint32_t)(st0 >> 48),
                              (uint32_t)(st1 & 0xFFFF), (uint32_t)((st1 >> 16) & 0xFFFF),
                              (uint32_t)((st1 >> 32) & 0xFFFF)};
    uint64_t tm = tmax1;
    for (int d = 32; d > 0; d >>= 1) tm = max(tm, (uint64_t)__shfl_xor(tm, d, 64));
    if (__lane_id() == 63) {
        w_cnt[w] = cinc;
        w_max[w] = minc;
    }
    if (__lane_id() == 0) {
        w_min[w] = fmin;
#pragma unroll
        for (int k = 0; k < 7; ++k) w_stat[w][k] = stat[k];
        w_stat[w][7] = tm;
    }
    uint32_t mex_w = __shfl_up(minc, 1, 64);
    if (__lane_id() == 0) mex_w = 0;
    __syncthreads();
    uint32_t tpre = cinc - nkeep, mex = mex_w, tile_keep = 0, tile_max1 = 0, tile_min = kNo;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        if (k < w) {
            tpre += w_cnt[k];
            mex = max(mex, w_max[k]);
        }
        tile_keep += w_cnt[k];
        tile_max1 = max(tile_max1, w_max[k]);
        tile_min = min(tile_min, w_min[k]);
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
                for (int q = 0; q < kWaves; ++q) v += w_stat[q][k];
                st[k] = v;
            }
            unsigned long long mx = 0;
            for (int q = 0; q < kWaves; ++q) mx = max(mx, w_stat[q][7]);
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
                for (int q = 0; q < kWaves; ++q) v += w_stat[q][k];
                if (v) atomicAdd(dst[k], v);
            }
            unsigned long long mx = 0;
            for (int q = 0; q < kWaves; ++q) mx = max(mx, w_stat[q][7]);
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
        for (int j = 0; j < kTileItems; ++j) {
            if (sv[j] != kNo) {
                if (o < a.ev_cap) {
                    const Word d = decode_word(sp[tile_slot(threadIdx.x * kTileItems + j)], a.sub);
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
        // kept events staged in LDS in output order, then written contiguously
        {
            uint32_t q = tpre;
#pragma unroll
            for (int j = 0; j < kTileItems; ++j)
                if (sv[j] != kNo) sp[tile_slot(q++)] = tv[j];
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < tile_keep; k += kTileThreads)
            if (out0 + k < a.ev_cap) a.ev[out0 + k] = sp[tile_slot(k)];
        if (a.shot_out) {
            __syncthreads();
            uint32_t q = tpre;
#pragma unroll
            for (int j = 0; j < kTileItems; ++j)
                if (sv[j] != kNo) sp[tile_slot(q++)] = sv[j];
            __syncthreads();
            for (uint32_t k = threadIdx.x; k < tile_keep; k += kTileThreads)
                if (out0 + k < a.ev_cap) a.shot_out[out0 + k] = (uint32_t)sp[tile_slot(k)];
        }
        // events per shot from run boundaries: a run of shot s over positions
        // [p, p') adds p' - p to its count.  Exact when the kept events are in
        // shot order (otherwise the caller takes the sorting path).
        if (a.shot_cnt && nkeep) {
            uint32_t prev = mex;  // previous kept shot in the tile + 1, 0 = none
            uint32_t p = (uint32_t)(pcount + tpre);
#pragma unroll
            for (int j = 0; j < kTileItems; ++j) {
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

// -------------------------------------------------------------- launchers
void launch_tile_summary(const uint64_t* pk, uint64_t n, uint32_t sub, uint64_t jump,
                         TileAcc* sums, uint64_t* tdc_slot, hipStream_t s) {
    const uint64_t ntiles = (n + kTilePkts - 1) / kTilePkts;
    if (ntiles == 0) return;
    hipLaunchKernelGGL(k_tile_summary, dim3((unsigned)ntiles), dim3(kSumThreads), 0, s, pk, n,
                       sub, jump, sums, tdc_slot);
}

uint64_t tile_scan_blocks(uint64_t ntiles) { return (ntiles + kScanTiles - 1) / kScanTiles; }

void launch_tile_scan(const TileAcc* sums, uint64_t ntiles, TileAcc init, int64_t pe0, int64_t te0,
                      uint64_t jump, TileAcc* partial, TileAcc* blk, DevResults* res,
                      hipStream_t s) {
    const uint64_t nblk = tile_scan_blocks(ntiles);
    if (nblk)
        hipLaunchKernelGGL(k_tile_scan1, dim3((unsigned)nblk), dim3(kScanTiles), 0, s, sums, ntiles,
                           jump, partial, blk);
    hipLaunchKernelGGL(k_tile_scan2, dim3(1), dim3(1024), 0, s, blk, nblk, init, pe0, te0, jump,
                       res);
}

void launch_trig_unwrap(const TileAcc* sums, const TileAcc* partial, const TileAcc* blk,
                        const uint64_t* slot, uint64_t ntiles, int64_t pe0, int64_t te0,
                        uint64_t jump, TileEntry* entries, uint64_t* tab, DevResults* res,
                        hipStream_t s) {
    if (ntiles == 0) return;
    hipLaunchKernelGGL(k_trig_unwrap, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s,
                       sums, partial, blk, slot, ntiles, tile_scan_blocks(ntiles), pe0, te0, jump,
                       entries, tab, res);
}

void launch_assign_staged(const AssignArgs& a, hipStream_t s) {
    const uint64_t ntiles = (a.n + kTilePkts - 1) / kTilePkts;
    if (ntiles == 0) return;
    hipLaunchKernelGGL((k_assign<false, true>), dim3((unsigned)ntiles), dim3(kTileThreads), 0, s,
                       a);
}

// Staged kept events of tile t to their place; the shot order across tiles
// (a tile's smallest kept shot below the largest of the nearest earlier tile
// with kept events, or of the carried events); the call's kept-event count.
constexpr int kPlaceThreads = 256;
__global__ __launch_bounds__(kPlaceThreads) void k_assign_place(AssignArgs a, const uint32_t* tile_off,
                                                                uint64_t* ev_out, uint64_t ev_off,
                                                                uint64_t ev_cap,
                                                                uint32_t* shot_final,
                                                                uint64_t ntiles) {
    const uint64_t t = blockIdx.x;
    if (t == 0 && threadIdx.x == 0) a.res->n_kept = tile_off[ntiles];
    const uint32_t cnt = a.tile_cnt[t];
    const uint64_t src = t * kTilePkts, dst = ev_off + tile_off[t];
    for (uint32_t k = threadIdx.x; k < cnt; k += kPlaceThreads) {
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

// Sum of the per-tile statistics (and the largest unwrapped time + 1).
constexpr int kStatBlocks = 64;
__global__ __launch_bounds__(256) void k_tile_stat_reduce(const unsigned long long* st, uint64_t ntiles,
                                                          DevResults* res) {
    __shared__ unsigned long long part[256 / 64][8];
    unsigned long long v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (uint64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] += st[8 * t + k];
        v[7] = max(v[7], st[8 * t + 7]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
        for (int d = 32; d > 0; d >>= 1) {
            const unsigned long long o = __shfl_xor(v[k], d, 64);
            v[k] = k < 7 ? v[k] + o : max(v[k], o);
        }
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0)
        for (int k = 0; k < 8; ++k) part[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 8) {
        const int k = threadIdx.x;
        unsigned long long x = 0;
        for (int q = 0; q < 256 / 64; ++q) x = k < 7 ? x + part[q][k] : max(x, part[q][k]);
        unsigned long long* dst[7] = {&res->n_pixels, &res->n_other, &res->n_pre_trigger,
                                      &res->n_tof_cut, &res->n_late_drop, &res->n_pix_wraps,
                                      &res->n_pix_backjumps};
        if (k < 7) {
            if (x) atomicAdd(dst[k], x);
        } else if (x) {
            atomicMax(&res->max_t_plus1, x);
        }
    }
}

void launch_assign_place(const AssignArgs& a, const uint32_t* tile_off, uint64_t* ev_out,
                         uint64_t ev_off, uint64_t ev_cap, uint32_t* shot_out_final,
                         hipStream_t s) {
    const uint64_t ntiles = (a.n + kTilePkts - 1) / kTilePkts;
    if (ntiles == 0) return;
    hipLaunchKernelGGL(k_assign_place, dim3((unsigned)ntiles), dim3(kPlaceThreads), 0, s, a,
                       tile_off, ev_out, ev_off, ev_cap, shot_out_final, ntiles);
    hipLaunchKernelGGL(k_tile_stat_reduce, dim3(kStatBlocks), dim3(256), 0, s, a.tile_stat, ntiles,
                       a.res);
}

void launch_assign(const AssignArgs& a, bool soa, hipStream_t s) {
    const uint64_t ntiles = (a.n + kTilePkts - 1) / kTilePkts;
    if (ntiles == 0) return;
    if (soa)
        hipLaunchKernelGGL(k_assign<true>, dim3((unsigned)ntiles), dim3(kTileThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_assign<false>, dim3((unsigned)ntiles), dim3(kTileThreads), 0, s, a);
}

}  // namespace tpx
