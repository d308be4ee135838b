// Device code of the stream path's bookkeeping (close rule, carry of open
// shots' events), shared by its kernels (tpx_util.hip) and the persistent
// chunk kernel.
#pragma once

#include "tpx_kernels.h"

namespace tpx {

// Shots [first_open, s_close) close in this chunk: trigger s+1 was seen and a
// word later than T[s] + tof_max + slack has arrived (everything on flush).
__device__ __forceinline__ void close_rule(const uint64_t* tab, const unsigned long long* n_trig_dev, uint64_t n_win,
                           uint64_t first_open, int flush, uint64_t max_t_plus1_prev,
                           uint64_t tof_max, uint64_t slack, const uint32_t* shot_off,
                           DevResults* res) {
    const uint64_t n_tab = n_win + *n_trig_dev;
    uint64_t s_close;
    if (flush) {
        s_close = n_tab;
    } else {
        uint64_t mt1 = max<uint64_t>(max_t_plus1_prev, res->max_t_plus1);
        if (n_tab) mt1 = max<uint64_t>(mt1, tab[n_tab - 1] + 1);
        uint64_t ub = 0;
        if (mt1 > tof_max + slack + 0) {
            const uint64_t lim = mt1 - 1 - tof_max - slack;  // T[s] <= lim closes s
            uint64_t lo = 0, hi = n_tab;
            while (lo < hi) {
                const uint64_t m = (lo + hi) >> 1;
                if (tab[m] <= lim) lo = m + 1; else hi = m;
            }
            ub = lo;
        }
        s_close = n_tab ? min<uint64_t>(ub, n_tab - 1) : 0;
        s_close = max<uint64_t>(s_close, min<uint64_t>(first_open, n_tab));
    }
    res->n_groups = n_tab;
    res->n_close_grp = s_close;
    res->n_close_ev = shot_off ? shot_off[s_close] : 0;
}
// the carried events i = first, first + stride, ... < n_carry.  The carried
// events are in shot order; when the lanes of a wave hold consecutive events
// (first = the thread's global index, stride a multiple of 64), each run of
// one shot within a wave adds its length with one atomic (the run's last
// lane), else every event adds one.
__device__ __forceinline__ void carry_in_range(const uint64_t* c_ev, const uint32_t* c_shot,
                                               uint64_t n_carry, uint32_t rebase, uint64_t* ev,
                                               uint32_t* shot_arr, uint32_t* shot_cnt,
                                               uint64_t first, uint64_t stride) {
    const bool runs = (stride & 63) == 0 && (first & 63) == __lane_id();
    for (uint64_t base = first - (first & 63); base < n_carry; base += stride) {
        const uint64_t i = base + (first & 63);
        const bool live = i < n_carry;
        uint32_t sidx = 0;
        if (live) {
            ev[i] = c_ev[i];
            sidx = c_shot[i] - rebase;
            if (shot_arr) shot_arr[i] = sidx;
        }
        if (!shot_cnt) continue;
        if (!runs) {
            if (live) atomicAdd(&shot_cnt[sidx], 1u);
            continue;
        }
        // lanes of this wave hold events base .. base + 63 (all lanes take
        // part, so the cross-lane reads are defined)
        const int lane = (int)__lane_id();
        const uint32_t next = __shfl_down(sidx, 1, 64);
        const bool last = live && (lane == 63 || i + 1 >= n_carry || next != sidx);
        const uint64_t ends = __ballot(last);
        const uint64_t below = ends & ((1ull << lane) - 1ull);
        const int start = below ? 64 - __clzll(below) : 0;
        if (last) atomicAdd(&shot_cnt[sidx], (uint32_t)(lane - start + 1));
    }
}

// events of the open shots, positions lo + first, lo + first + stride, ...
__device__ __forceinline__ void carry_out_range(const uint64_t* ev, const uint32_t* perm, const uint32_t* shot_arr,
                                const uint32_t* shot_off, const unsigned long long* n_rows_dev,
                                const unsigned long long* n_close_ev,
                                const unsigned long long* n_kept, const uint64_t* carry_gidx_in,
                                uint64_t n_carry, uint64_t ev_base, uint64_t* c_ev,
                                uint32_t* c_shot, uint64_t* c_gidx, uint64_t carry_cap,
                                DevResults* res, uint64_t first, uint64_t stride) {
    const uint64_t lo = *n_close_ev;
    const uint64_t hi = n_carry + *n_kept;
    if (hi > lo && hi - lo > carry_cap) {
        if (first == 0) atomicOr(&res->err, (unsigned long long)kErrCapacity);
        return;
    }
    const uint64_t rows = n_rows_dev ? *n_rows_dev : 0;
    for (uint64_t p = lo + first; p < hi; p += stride) {
        const uint64_t j = p - lo;
        c_ev[j] = ev[p];
        uint32_t sidx;
        if (shot_arr) {
            sidx = shot_arr[p];
        } else {  // last row g with shot_off[g] <= p
            uint64_t a = 0, b = rows;
            while (b - a > 1) {
                const uint64_t m = (a + b) >> 1;
                if (shot_off[m] <= p) a = m; else b = m;
            }
            sidx = (uint32_t)a;
        }
        c_shot[j] = sidx;
        if (p == hi - 1) res->carry_last = (unsigned long long)sidx + 1;
        const uint64_t o = perm ? perm[p] : p;
        c_gidx[j] = o < n_carry ? carry_gidx_in[o] : ev_base + (o - n_carry);
    }
}

}  // namespace tpx
