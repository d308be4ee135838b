// Decode, unwrap and shot assignment (Sec. III; Sec. IV, ToA Unwrapping and
// Eliminating Background Counts) as three passes over 4096-word tiles:
//   k_tile_summary  per tile: folded pixel / trigger counter runs and the
//                   trigger words in stream order (one read of the packets);
//   k_tile_scan     one workgroup folds the tile summaries into the state in
//                   force at the start of every tile;
//   k_trig_unwrap   unwraps the trigger words into the trigger table;
//   k_assign        second read of the packets: unwraps each pixel, finds its
//                   shot (latest trigger at or before it), applies the ToF
//                   cut and writes the kept events in stream order (stable
//                   compaction with a decoupled look-back over tiles).
#include "tpx_kernels.h"

namespace tpx {

// Packets of one tile staged through LDS so that each thread can walk 16
// consecutive words: padded by one word per 16 to spread LDS banks.
__device__ inline int tile_slot(int i) { return i + (i >> 4); }
constexpr int kTileLds = kTilePkts + kTilePkts / 16;

__device__ inline void load_tile(const uint64_t* __restrict__ pk, uint64_t base, uint64_t n,
                                 uint64_t* sp) {
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        const int i = k * kTileThreads + threadIdx.x;
        const uint64_t g = base + (uint64_t)i;
        sp[tile_slot(i)] = g < n ? __builtin_nontemporal_load(pk + g) : 0ull;
    }
}

// Exclusive in-order fold of one RunSum per thread (256 threads) through LDS.
// Returns the fold of all threads before the caller; *all gets the total.
__device__ inline RunSum wg_run_exscan(RunSum v, RunSum* buf, uint64_t jump, RunSum* all) {
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    if (t < 64) {  // each lane folds 4 consecutive entries, lane 0 folds lanes
        RunSum a = run_empty();
        for (int k = 0; k < 4; ++k) a = run_combine(a, buf[t * 4 + k], jump);
        buf[256 + t] = a;
    }
    __syncthreads();
    if (t == 0) {
        RunSum a = run_empty();
        for (int k = 0; k < 64; ++k) {
            const RunSum c = buf[256 + k];
            buf[256 + k] = a;  // exclusive
            a = run_combine(a, c, jump);
        }
        buf[320] = a;
    }
    __syncthreads();
    RunSum pre = buf[256 + (t >> 2)];
    for (int k = (t & ~3); k < t; ++k) pre = run_combine(pre, buf[k], jump);
    *all = buf[320];
    __syncthreads();
    return pre;
}

__global__ __launch_bounds__(kTileThreads) void k_tile_summary(const uint64_t* __restrict__ pk,
                                                              uint64_t n, uint32_t sub,
                                                              uint64_t jump, TileSum* sums,
                                                              uint64_t* tdc_slot,
                                                              uint32_t* tdc_cnt) {
    __shared__ uint64_t sp[kTileLds];
    __shared__ RunSum buf[321];
    __shared__ uint32_t tmp[kTileThreads / 64 + 1];
    const uint64_t tile = blockIdx.x;
    const uint64_t base = tile * kTilePkts;
    load_tile(pk, base, n, sp);
    __syncthreads();
    const int nvalid = (int)min<uint64_t>((uint64_t)kTilePkts, n - base);
    RunSum P = run_empty(), T = run_empty();
    uint32_t nt = 0;
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
        const int i = threadIdx.x * kTileItems + j;
        if (i < nvalid) {
            const Word d = decode_word(sp[tile_slot(i)], sub);
            if (d.kind == kPixel) {
                P = run_combine(P, RunSum{d.raw, d.raw, 0, 1}, jump);
            } else if (d.kind == kTrigger) {
                T = run_combine(T, RunSum{d.raw, d.raw, 0, 1}, jump);
                ++nt;
            }
        }
    }
    uint32_t ntot;
    const uint32_t pos = wg_count_scan<kTileThreads>(nt, tmp, &ntot);
    if (nt) {
        uint32_t q = 0;
        for (int j = 0; j < kTileItems; ++j) {
            const int i = threadIdx.x * kTileItems + j;
            if (i < nvalid) {
                const Word d = decode_word(sp[tile_slot(i)], sub);
                if (d.kind == kTrigger) tdc_slot[base + pos + q++] = d.raw;
            }
        }
    }
    RunSum ap, at;
    wg_run_exscan(P, buf, jump, &ap);
    wg_run_exscan(T, buf, jump, &at);
    if (threadIdx.x == 0) {
        sums[tile].pix = ap;
        sums[tile].tdc = at;
        tdc_cnt[tile] = ntot;
    }
}

// One workgroup of 1024 threads folds all tile summaries in order.
__global__ __launch_bounds__(1024) void k_tile_scan(const TileSum* __restrict__ sums,
                                                   const uint32_t* __restrict__ tdc_cnt,
                                                   uint64_t ntiles, RunSum pix0, RunSum tdc0,
                                                   int64_t pix_epoch0, int64_t tdc_epoch0,
                                                   uint64_t jump, TileEntry* entries,
                                                   DevResults* res) {
    __shared__ TileSum agg[1024];
    __shared__ uint64_t cnt[1024];
    __shared__ TileSum grp[65];
    __shared__ uint64_t gcnt[65];
    const int t = threadIdx.x;
    const uint64_t per = (ntiles + 1023) / 1024;
    const uint64_t lo = min<uint64_t>(ntiles, (uint64_t)t * per);
    const uint64_t hi = min<uint64_t>(ntiles, lo + per);
    TileSum a{run_empty(), run_empty()};
    uint64_t c = 0;
    for (uint64_t k = lo; k < hi; ++k) {
        a.pix = run_combine(a.pix, sums[k].pix, jump);
        a.tdc = run_combine(a.tdc, sums[k].tdc, jump);
        c += tdc_cnt[k];
    }
    agg[t] = a;
    cnt[t] = c;
    __syncthreads();
    if (t < 64) {
        TileSum g{run_empty(), run_empty()};
        uint64_t gc = 0;
        for (int k = 0; k < 16; ++k) {
            const TileSum& e = agg[t * 16 + k];
            g.pix = run_combine(g.pix, e.pix, jump);
            g.tdc = run_combine(g.tdc, e.tdc, jump);
            gc += cnt[t * 16 + k];
        }
        grp[t] = g;
        gcnt[t] = gc;
    }
    __syncthreads();
    if (t == 0) {
        TileSum run{pix0, tdc0};
        uint64_t rc = 0;
        for (int k = 0; k < 64; ++k) {
            const TileSum g = grp[k];
            const uint64_t gc = gcnt[k];
            grp[k] = run;
            gcnt[k] = rc;
            run.pix = run_combine(run.pix, g.pix, jump);
            run.tdc = run_combine(run.tdc, g.tdc, jump);
            rc += gc;
        }
        grp[64] = run;
        gcnt[64] = rc;
    }
    __syncthreads();
    TileSum pre = grp[t >> 4];
    uint64_t pc = gcnt[t >> 4];
    for (int k = t & ~15; k < t; ++k) {
        pre.pix = run_combine(pre.pix, agg[k].pix, jump);
        pre.tdc = run_combine(pre.tdc, agg[k].tdc, jump);
        pc += cnt[k];
    }
    for (uint64_t k = lo; k < hi; ++k) {
        TileEntry e;
        e.pix = pre.pix;
        e.tdc = pre.tdc;
        e.pix_epoch = pix_epoch0 + pre.pix.sum;
        e.tdc_epoch = tdc_epoch0 + pre.tdc.sum;
        e.trig_off = pc;
        entries[k] = e;
        pre.pix = run_combine(pre.pix, sums[k].pix, jump);
        pre.tdc = run_combine(pre.tdc, sums[k].tdc, jump);
        pc += tdc_cnt[k];
    }
    if (t == 0) {
        const TileSum all = grp[64];
        res->pix_epoch_end = pix_epoch0 + all.pix.sum;
        res->tdc_epoch_end = tdc_epoch0 + all.tdc.sum;
        res->pix_last_end = all.pix.last;
        res->tdc_last_end = all.tdc.last;
        res->pix_has_end = all.pix.count > 0;
        res->tdc_has_end = all.tdc.count > 0;
        res->n_trig = gcnt[64];
    }
}

// One thread per tile unwraps that tile's trigger words in order.
__global__ void k_trig_unwrap(const TileEntry* __restrict__ entries,
                              const uint32_t* __restrict__ tdc_cnt,
                              const uint64_t* __restrict__ tdc_slot, uint64_t ntiles,
                              uint64_t jump, uint64_t* tab, DevResults* res) {
    const uint64_t tile = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    const uint32_t c = tdc_cnt[tile];
    if (c == 0) return;
    const TileEntry e = entries[tile];
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

template <bool kSoA>
__global__ __launch_bounds__(kTileThreads) void k_assign(AssignArgs a) {
    __shared__ uint64_t sp[kTileLds];
    __shared__ RunSum buf[321];
    __shared__ uint64_t slice[kTrigSlice];
    __shared__ uint32_t tmp[kTileThreads / 64 + 1];
    __shared__ uint64_t bcast[8];
    __shared__ uint32_t gmin_s[kTileThreads], gmax_s[kTileThreads];
    __shared__ uint32_t unsorted_s;

    if (threadIdx.x == 0) {
        bcast[0] = atomicAdd(&a.res->tile_ticket, 1ull);
        unsorted_s = 0;
    }
    __syncthreads();
    const uint64_t tile = bcast[0];
    const uint64_t base = tile * kTilePkts;
    load_tile(a.pk, base, a.n, sp);
    __syncthreads();
    const int nvalid = (int)min<uint64_t>((uint64_t)kTilePkts, a.n - base);
    const TileEntry e = a.entries[tile];
    const uint64_t n_tab = a.n_win + *a.n_trig_dev;

    // this thread's run of pixel counter values, folded across the workgroup
    RunSum P = run_empty();
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
        const int i = threadIdx.x * kTileItems + j;
        if (i < nvalid) {
            const Word d = decode_word(sp[tile_slot(i)], a.sub);
            if (d.kind == kPixel) P = run_combine(P, RunSum{d.raw, d.raw, 0, 1}, a.jump);
        }
    }
    RunSum all;
    const RunSum pre = run_combine(e.pix, wg_run_exscan(P, buf, a.jump, &all), a.jump);

    // unwrap this thread's pixels
    uint64_t tv[kTileItems];
    bool has = pre.count > 0;
    uint64_t last = pre.last;
    int64_t epoch = e.pix_epoch + (pre.sum - e.pix.sum);
    uint64_t tmin = ~0ull, tmax = 0;
    unsigned long long fwd = 0, back = 0, npix = 0, nother = 0, err = 0;
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
        const int i = threadIdx.x * kTileItems + j;
        tv[j] = ~0ull;
        if (i < nvalid) {
            const Word d = decode_word(sp[tile_slot(i)], a.sub);
            if (d.kind == kPixel) {
                if (has) {
                    const int jj = jump_of(last, d.raw, a.jump);
                    epoch += jj;
                    fwd += jj > 0;
                    back += jj < 0;
                }
                has = true;
                last = d.raw;
                ++npix;
                if (epoch < 0) {
                    err |= kErrStream;
                } else {
                    tv[j] = d.raw + (uint64_t)epoch * kPixPeriod;
                    tmin = min(tmin, tv[j]);
                    tmax = max(tmax, tv[j]);
                }
            } else if (d.kind == kOther) {
                ++nother;
            }
        }
    }

    // time range of the tile's pixels -> slice of the trigger table in LDS
    {
        uint64_t mn = tmin, mx = tmax;
        for (int d = 32; d > 0; d >>= 1) {
            mn = min(mn, (uint64_t)__shfl_xor(mn, d, 64));
            mx = max(mx, (uint64_t)__shfl_xor(mx, d, 64));
        }
        if (__lane_id() == 0) {
            reinterpret_cast<uint64_t*>(gmin_s)[threadIdx.x >> 6] = mn;
            reinterpret_cast<uint64_t*>(gmax_s)[threadIdx.x >> 6] = mx;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < kTileThreads / 64; ++w) {
                mn = min(mn, reinterpret_cast<uint64_t*>(gmin_s)[w]);
                mx = max(mx, reinterpret_cast<uint64_t*>(gmax_s)[w]);
            }
            uint64_t s_lo = 0, s_hi = 0, use = 0;
            if (mn <= mx && n_tab > 0) {
                const uint64_t ulo = upper_bound_u64(a.tab, 0, n_tab, mn);
                const uint64_t uhi = upper_bound_u64(a.tab, ulo, n_tab, mx);
                s_lo = ulo > 0 ? ulo - 1 : 0;
                s_hi = uhi;  // exclusive end of the candidate shots + 1
                if (s_hi - s_lo <= (uint64_t)kTrigSlice) use = 1;
            }
            bcast[1] = s_lo;
            bcast[2] = s_hi;
            bcast[3] = use;
        }
        __syncthreads();
    }
    const uint64_t s_lo = bcast[1], s_hi = bcast[2];
    const bool use_slice = bcast[3] != 0;
    if (use_slice) {
        for (uint64_t k = threadIdx.x; k < s_hi - s_lo; k += kTileThreads) slice[k] = a.tab[s_lo + k];
    }
    __syncthreads();

    // shot of each pixel, cut, keep
    uint32_t sv[kTileItems];
    uint32_t nkeep = 0;
    unsigned long long npre = 0, ncut = 0, nlate = 0;
    uint32_t first_s = 0xFFFFFFFFu, last_s = 0;
    bool sorted = true;
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
        sv[j] = 0xFFFFFFFFu;
        if (tv[j] != ~0ull) {
            const uint64_t t = tv[j];
            uint64_t ub;
            if (use_slice) {
                ub = s_lo + upper_bound_u64(slice, 0, s_hi - s_lo, t);
                if (ub == s_lo && s_lo > 0) ub = upper_bound_u64(a.tab, 0, s_lo, t);
            } else {
                ub = upper_bound_u64(a.tab, 0, n_tab, t);
            }
            if (ub == 0) {
                if (a.tab_has_before) ++nlate; else ++npre;
            } else {
                const uint64_t s = ub - 1;
                const uint64_t tof = t - a.tab[s];
                if (tof > a.tof_max) {
                    ++ncut;
                } else if (s < a.first_open) {
                    ++nlate;
                } else {
                    sv[j] = (uint32_t)s;
                    ++nkeep;
                    if (first_s == 0xFFFFFFFFu) first_s = (uint32_t)s;
                    if ((uint32_t)s < last_s) sorted = false;
                    last_s = (uint32_t)s;
                }
            }
        }
    }

    // stable compaction: thread prefix, tile total, look-back over tiles
    uint32_t tile_keep;
    const uint32_t tpre = wg_count_scan<kTileThreads>(nkeep, tmp, &tile_keep);
    if (threadIdx.x == 0) {
        if (tile == 0) {
            lb_publish(a.lb_status, 0, kLbInclusive, tile_keep);
            bcast[4] = 0;
        } else {
            lb_publish(a.lb_status, tile, kLbAggregate, tile_keep);
            const uint64_t p = lb_lookback(a.lb_status, tile, &a.res->err);
            lb_publish(a.lb_status, tile, kLbInclusive, p + tile_keep);
            bcast[4] = p;
        }
    }
    // order check across threads: a thread's first kept shot must not be
    // below the last kept shot of any earlier thread
    gmin_s[threadIdx.x] = nkeep ? first_s : 0xFFFFFFFFu;
    gmax_s[threadIdx.x] = nkeep ? last_s : 0u;
    if (!sorted) atomicOr(&unsorted_s, 1u);
    __syncthreads();
    const uint64_t out0 = a.ev_off + bcast[4] + tpre;
    if (threadIdx.x == 0) {
        uint32_t run_max = 0, any = 0, f = 0xFFFFFFFFu;
        bool ok = true;
        for (int k = 0; k < kTileThreads; ++k) {
            if (gmin_s[k] == 0xFFFFFFFFu) continue;
            if (any && gmin_s[k] < run_max) ok = false;
            if (!any) f = gmin_s[k];
            any = 1;
            run_max = max(run_max, gmax_s[k]);
        }
        if (a.recs) {
            TileRec r;
            r.first_g = f;
            r.last_g = run_max;
            r.n_kept = tile_keep;
            r.sorted = (ok && unsorted_s == 0) ? 1u : 0u;
            a.recs[tile] = r;
        }
    }

    // write kept events in stream order; count events per shot
    uint64_t o = out0;
    uint32_t run_s = 0xFFFFFFFFu, run_n = 0;
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
        if (sv[j] != 0xFFFFFFFFu) {
            const int i = threadIdx.x * kTileItems + j;
            const Word d = decode_word(sp[tile_slot(i)], a.sub);
            const uint64_t s = sv[j];
            if (o < a.ev_cap) {
                if constexpr (kSoA) {
                    a.soa.x[o] = (uint16_t)d.x;
                    a.soa.y[o] = (uint16_t)d.y;
                    a.soa.tot[o] = (uint16_t)d.tot;
                    a.soa.shot[o] = (uint32_t)(a.shot_base + s);
                    a.soa.toa[o] = tv[j];
                } else {
                    a.ev[o] = pack_event(d.x, d.y, d.tot, (uint32_t)(tv[j] - a.tab[s]));
                    if (a.shot_out) a.shot_out[o] = (uint32_t)s;
                }
            }
            ++o;
            if (a.shot_cnt) {
                if ((uint32_t)s != run_s) {
                    if (run_n) atomicAdd(&a.shot_cnt[run_s], run_n);
                    run_s = (uint32_t)s;
                    run_n = 0;
                }
                ++run_n;
            }
        }
    }
    if (a.shot_cnt && run_n) atomicAdd(&a.shot_cnt[run_s], run_n);

    // statistics
    const unsigned long long vals[7] = {npix, nother, npre, ncut, nlate, fwd, back};
    unsigned long long* dst[7] = {&a.res->n_pixels, &a.res->n_other, &a.res->n_pre_trigger,
                                  &a.res->n_tof_cut, &a.res->n_late_drop, &a.res->n_pix_wraps,
                                  &a.res->n_pix_backjumps};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        unsigned long long v = vals[k];
        for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
        if (__lane_id() == 0 && v) atomicAdd(dst[k], v);
    }
    {
        uint64_t mx = tmax;
        if (tmin > tmax) mx = 0;
        for (int d = 32; d > 0; d >>= 1) mx = max(mx, (uint64_t)__shfl_xor(mx, d, 64));
        if (__lane_id() == 0 && mx) atomicMax(&a.res->max_t_plus1, (unsigned long long)(mx + 1));
    }
    if (err) atomicOr(&a.res->err, err);
    if (threadIdx.x == 0) atomicAdd(&a.res->n_kept, (unsigned long long)tile_keep);
}

// -------------------------------------------------------------- launchers
void launch_tile_summary(const uint64_t* pk, uint64_t n, uint32_t sub, uint64_t jump,
                         TileSum* sums, uint64_t* tdc_slot, uint32_t* tdc_cnt, hipStream_t s) {
    const uint64_t ntiles = (n + kTilePkts - 1) / kTilePkts;
    if (ntiles == 0) return;
    hipLaunchKernelGGL(k_tile_summary, dim3((unsigned)ntiles), dim3(kTileThreads), 0, s, pk, n,
                       sub, jump, sums, tdc_slot, tdc_cnt);
}

void launch_tile_scan(const TileSum* sums, const uint32_t* tdc_cnt, uint64_t ntiles, RunSum pix0,
                      RunSum tdc0, int64_t pe0, int64_t te0, uint64_t jump, TileEntry* entries,
                      DevResults* res, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, sums, tdc_cnt, ntiles, pix0, tdc0,
                       pe0, te0, jump, entries, res);
}

void launch_trig_unwrap(const TileEntry* entries, const uint32_t* tdc_cnt, const uint64_t* slot,
                        uint64_t ntiles, uint64_t jump, uint64_t* tab, DevResults* res,
                        hipStream_t s) {
    if (ntiles == 0) return;
    hipLaunchKernelGGL(k_trig_unwrap, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s,
                       entries, tdc_cnt, slot, ntiles, jump, tab, res);
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
