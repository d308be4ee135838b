// Connectivity clustering and ToT-weighted centroids (Sec. V: Neighborhoods,
// Eqs. 3-5, closed transitively; Centroiding, Eqs. 8-9).
//
// Events arrive grouped by shot.  Groups are packed into segments of about
// `q` events and every workgroup clusters one segment.  Workgroups take their
// segment from an atomic ticket, so that segment k's workgroup started after
// those of segments 0..k-1; a decoupled look-back over segments then gives
// each segment its first output slot.  Inside a segment:
//   1. every event is dropped into a hashed 256x64 image of its pixel address
//      (LDS); events sharing an image slot are chained behind the slot owner;
//   2. each event visits the slots of its forward neighbourhood (the half of
//      the (2r+1)^2 box that comes after it, plus its own slot) and unites
//      with every chained event that has the same shot, |dx|,|dy| <= r and
//      |dt| <= r_t: the edges of the paper's Hadamard adjacency A;
//   3. a lock-free union-find in LDS, always hooking the larger root under the
//      smaller, leaves every component rooted at its smallest event position,
//      which is also its smallest event index;
//   4. ToT-weighted integer moments are accumulated per root with LDS atomics
//      (exact, so the result does not depend on the order of the atomics) and
//      each root emits one hit: X = sum(ToT x)/sum(ToT), same for Y and ToF.
// Segments larger than the LDS capacity take the same steps with their
// per-event arrays in global memory.  Control flow around every barrier is
// uniform: one segment per workgroup, a fixed sequence of phases.
#include "tpx_kernels.h"

namespace tpx {

constexpr int kCap = 2048;             // events per segment held in LDS
constexpr int kWG = 512;               // threads per workgroup
constexpr int kK = kCap / kWG;         // events per thread
constexpr int kH = 16384;              // image slots: (y & 63) << 8 | x
constexpr uint32_t kNone32 = 0xFFFFFFFFu;
constexpr uint32_t kNone16 = 0xFFFFu;

// LDS byte layout of the small-segment path
constexpr int kOffImg = 0;             // u16[kH]
constexpr int kOffPar = 32768;         // u32[kCap] union-find parent
constexpr int kOffChn = 40960;         // u32[kCap] first chained event of a slot owner
constexpr int kOffT = 49152;           // u32[kCap] time (ticks after the shot reference)
constexpr int kOffSl = 57344;          // u32[kCap] group (shot) of the event
constexpr int kOffXy = 65536;          // u16[kCap] x | y << 8
constexpr int kOffNxt = 69632;         // u16[kCap] next chained event
constexpr int kLdsMain = 73728;
// accumulators overlaid on the same bytes once the components are known
constexpr int kOffW = 0, kOffSx = 8192, kOffSy = 16384, kOffCnt = 24576, kOffTmin = 32768,
              kOffSt = 40960;  // u64[kCap]
static_assert(kOffSt + 8 * kCap <= kLdsMain, "accumulator overlay");
static_assert(4 * kH <= kLdsMain, "big-path image");

__device__ inline uint32_t slot_of(uint32_t x, uint32_t y) { return ((y & 63u) << 8) | x; }
__device__ inline uint32_t absdiff(uint32_t a, uint32_t b) { return a > b ? a - b : b - a; }

// Words that several threads of the workgroup touch at once are read and
// written through relaxed workgroup-scope atomics.
__device__ inline uint32_t ald(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void ast(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Union-find with parent[v] <= v; roots satisfy parent[v] == v.  Every walk
// is bounded by the number of elements `lim`: a longer walk can only come from
// corrupted state, and is reported instead of spinning.
__device__ inline uint32_t uf_find(uint32_t* par, uint32_t v, uint32_t lim,
                                   unsigned long long* err) {
    uint32_t p = ald(par + v);
    if (p != v) {
        uint32_t prev = v, nx;
        uint32_t steps = 0;
        while (p > (nx = ald(par + p))) {
            ast(par + prev, nx);  // path halving; only ever moves towards the root
            prev = p;
            p = nx;
            if (++steps > lim) {
                atomicOr(err, (unsigned long long)kErrLoopFind);
                break;
            }
        }
    }
    return p;
}

__device__ inline void uf_unite(uint32_t* par, uint32_t a, uint32_t b, uint32_t lim,
                                unsigned long long* err) {
    uint32_t ra = uf_find(par, a, lim, err), rb = uf_find(par, b, lim, err);
    uint32_t tries = 0;
    while (ra != rb) {
        if (ra < rb) {
            const uint32_t t = ra;
            ra = rb;
            rb = t;
        }
        // hook the larger root ra under the smaller root rb
        uint32_t expect = ra;
        if (__hip_atomic_compare_exchange_strong(par + ra, &expect, rb, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            break;
        if (++tries > 2 * lim + 2) {
            atomicOr(err, (unsigned long long)kErrLoopUnite);
            break;
        }
        ra = uf_find(par, expect, lim, err);
        rb = uf_find(par, rb, lim, err);
    }
}

struct Ev {
    uint32_t x, y, tot, t, g;
    uint64_t pos;  // position in the sorted event order
};

// group (shot) of sorted position p: last g in [lo, hi) with off[g] <= p
template <typename P>
__device__ inline uint32_t group_of(P off, uint32_t lo, uint32_t hi, uint32_t p) {
    while (hi - lo > 1) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (off[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

template <bool kEvent>
__device__ inline bool load_event(const ClusterArgs& a, uint64_t p, const uint32_t* goff, uint32_t goff_base,
                                  uint32_t ng, bool goff_lds, uint32_t g_lo, Ev& e,
                                  unsigned long long* err) {
    e.pos = p;
    const uint32_t g = goff_lds ? g_lo + group_of(goff, 0, ng, (uint32_t)p)
                                : group_of(a.grp_off, g_lo, g_lo + ng, (uint32_t)p);
    (void)goff_base;
    e.g = g;
    if constexpr (!kEvent) {
        const uint64_t pk = a.ev[p];
        e.x = ev_x(pk);
        e.y = ev_y(pk);
        e.tot = ev_tot(pk);
        e.t = ev_t(pk);
    } else {
        const uint64_t o = a.perm ? a.perm[p] : p;
        e.x = a.soa.x[o];
        e.y = a.soa.y[o];
        e.tot = 0;
        const uint64_t first = a.grp_off[g];
        const uint64_t of = a.perm ? a.perm[first] : first;
        const uint64_t d = a.soa.toa[o] - a.soa.toa[of] + (1ull << 31);
        if (e.x > 255u || e.y > 255u || d >= (1ull << 32)) {
            atomicOr(err, (unsigned long long)kErrInput);
            e.x &= 255u;
            e.y &= 255u;
        }
        e.t = (uint32_t)d;
    }
    return true;
}

// global event index of sorted position p (stream path)
__device__ inline uint64_t gidx_of(const ClusterArgs& a, uint64_t p) {
    const uint64_t o = a.perm ? a.perm[p] : p;
    return o < a.n_carry ? a.carry_gidx[o] : a.ev_base + (o - a.n_carry);
}

__device__ inline uint64_t orig_of(const ClusterArgs& a, uint64_t p) {
    return a.perm ? a.perm[p] : p;
}

// St term of one pixel: ticks (no walk table) or 2^-16 ns fixed point
__device__ inline uint64_t time_term(const ClusterArgs& a, uint32_t tot, uint32_t t) {
    if (a.walk) {
        const int64_t wq = llrint((double)a.walk[tot & 1023u] * 65536.0);
        return (uint64_t)((int64_t)tot * ((int64_t)t * 102400 - wq));
    }
    return (uint64_t)tot * t;
}
__device__ inline uint64_t time_term1(const ClusterArgs& a, uint32_t tot, uint32_t t) {
    if (a.walk) {
        const int64_t wq = llrint((double)a.walk[tot & 1023u] * 65536.0);
        return (uint64_t)((int64_t)t * 102400 - wq);
    }
    return t;
}

__device__ inline void write_hit(const ClusterArgs& a, uint64_t h, uint32_t g, uint64_t W,
                                 uint64_t cnt, uint64_t sx, uint64_t sy, uint64_t st,
                                 uint32_t tmin, uint64_t label) {
    if (h >= a.hit_cap) return;
    const uint32_t sw = a.grp_shot ? a.grp_shot[g] : g;
    tpx_hit o;
    const double den = W ? (double)W : (double)cnt;
    o.x = (float)((double)sx / den);
    o.y = (float)((double)sy / den);
    const double num = a.walk ? (double)(int64_t)st * (1.0 / 65536.0) : 1.5625 * (double)st;
    o.tof_ns = (float)(num / den);
    o.npix = (uint32_t)cnt;
    o.shot = a.tab_base + sw;
    o.label = label;
    o.toa_first = a.tab[sw] + tmin;
    o.tot_sum = (uint32_t)W;
    o.flags = W ? 0u : 1u;
    a.hits[h] = o;
}

// Look-back over segments by the 64 lanes of wave 0; returns this segment's
// first output slot.
__device__ inline uint64_t seg_lookback(const ClusterArgs& a, uint64_t ticket, uint32_t count) {
    uint64_t p = 0;
    if (ticket > 0) {
        if (__lane_id() == 0) lb_publish(a.lb_status, ticket, kLbAggregate, count);
        p = lb_lookback_wave<LbSum>(a.lb_status, ticket, &a.res->err);
    }
    if (__lane_id() == 0) lb_publish(a.lb_status, ticket, kLbInclusive, p + count);
    return p;
}

// Visit every chained event of image slot (nx, ny) that is a neighbour of
// event i (same shot, |dx|, |dy| <= r, |dt| <= dt) and unite with it.  On the
// event's own slot only smaller positions are taken, so each pair is seen once.
template <typename IMG, typename NXT, typename XY>
__device__ inline void visit_slot(IMG img, uint32_t* chn, NXT nxt, const uint32_t* tt,
                                  const uint32_t* sl, XY xy, uint32_t* par, uint32_t i, int x, int y, uint32_t t, uint32_t g,
                                  int nx, int ny, bool own, int r, uint32_t dt, uint32_t n,
                                  uint32_t empty, unsigned long long* err) {
    const uint32_t w = img[slot_of((uint32_t)nx, (uint32_t)ny)];
    if (w == empty) return;
    uint32_t j = w;
    uint32_t link = chn[w];
    uint32_t steps = 0;
    while (true) {
        if (j != i && (!own || j < i)) {
            const uint32_t v = xy[j];
            const int xj = (int)(v & 255u), yj = (int)((v >> 8) & 255u);
            if (sl[j] == g && absdiff(tt[j], t) <= dt && abs(xj - x) <= r && abs(yj - y) <= r)
                uf_unite(par, i, j, n, err);
        }
        if (link == kNone32) break;
        if (++steps > n) {
            atomicOr(err, (unsigned long long)kErrLoopChain);
            break;
        }
        j = link;
        const uint32_t nn = nxt[j];
        link = (nn == empty) ? kNone32 : nn;
    }
}

// ------------------------------------------------------------ LDS segment
template <bool kEvent>
__device__ void seg_small(const ClusterArgs& a, uint8_t* lds, uint32_t* scan_tmp, uint64_t* bc,
                          const uint32_t* goff, bool goff_lds, uint32_t g_lo, uint32_t ng,
                          uint64_t e0, uint32_t n, uint64_t ticket) {
    uint16_t* img = (uint16_t*)(lds + kOffImg);
    uint32_t* par = (uint32_t*)(lds + kOffPar);
    uint32_t* chn = (uint32_t*)(lds + kOffChn);
    uint32_t* tt = (uint32_t*)(lds + kOffT);
    uint32_t* sl = (uint32_t*)(lds + kOffSl);
    uint16_t* xy = (uint16_t*)(lds + kOffXy);
    uint16_t* nxt = (uint16_t*)(lds + kOffNxt);
    const int tid = threadIdx.x;
    const int r = (int)a.dxy;
    const uint32_t dt = a.dt;
    unsigned long long* err = &a.res->err;

    // image of empty slots
    {
        uint4* v = (uint4*)img;
        for (int i = tid; i < kH * 2 / 16; i += kWG) v[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
    }
    Ev ev[kK];
    uint32_t root[kK];
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const uint32_t i = tid + k * kWG;
        if (i < n) {
            load_event<kEvent>(a, e0 + i, goff, 0, ng, goff_lds, g_lo, ev[k], err);
            par[i] = i;
            chn[i] = kNone32;
            tt[i] = ev[k].t;
            sl[i] = ev[k].g;
            xy[i] = (uint16_t)(ev[k].x | (ev[k].y << 8));
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const uint32_t i = tid + k * kWG;
        if (i < n) img[slot_of(ev[k].x, ev[k].y)] = (uint16_t)i;
    }
    __syncthreads();
    // events that lost the race for their slot chain behind the owner
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const uint32_t i = tid + k * kWG;
        if (i < n) {
            const uint32_t w = img[slot_of(ev[k].x, ev[k].y)];
            if (w != i) {
                const uint32_t old = atomicExch(&chn[w], i);
                nxt[i] = (uint16_t)(old == kNone32 ? kNone16 : old);
            }
        }
    }
    __syncthreads();
    // edges of the neighbourhood graph
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const uint32_t i = tid + k * kWG;
        if (i < n) {
            const int x = (int)ev[k].x, y = (int)ev[k].y;
            for (int dy = 0; dy <= r; ++dy) {
                const int ny = y + dy;
                if (ny > 255) break;
                for (int dx = (dy == 0 ? 0 : -r); dx <= r; ++dx) {
                    const int nx = x + dx;
                    if (nx < 0 || nx > 255) continue;
                    visit_slot(img, chn, nxt, tt, sl, xy, par, i, x, y,
                               ev[k].t, ev[k].g, nx, ny, dx == 0 && dy == 0, r, dt, n, kNone16,
                               err);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const uint32_t i = tid + k * kWG;
        root[k] = i < n ? uf_find(par, i, n, err) : 0u;
    }
    __syncthreads();

    if constexpr (kEvent) {
        uint32_t nroot = 0;
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            const uint32_t i = tid + k * kWG;
            if (i < n) {
                a.labels[orig_of(a, e0 + i)] = (uint32_t)orig_of(a, e0 + root[k]);
                nroot += root[k] == i;
            }
        }
        for (int d = 32; d > 0; d >>= 1) nroot += __shfl_xor(nroot, d, 64);
        if (__lane_id() == 0 && nroot) atomicAdd(&a.res->n_hits, (unsigned long long)nroot);
    } else {
        uint32_t* W = (uint32_t*)(lds + kOffW);
        uint32_t* SX = (uint32_t*)(lds + kOffSx);
        uint32_t* SY = (uint32_t*)(lds + kOffSy);
        uint32_t* CNT = (uint32_t*)(lds + kOffCnt);
        uint32_t* TMIN = (uint32_t*)(lds + kOffTmin);
        unsigned long long* ST = (unsigned long long*)(lds + kOffSt);
        for (uint32_t i = tid; i < n; i += kWG) {
            W[i] = 0;
            SX[i] = 0;
            SY[i] = 0;
            CNT[i] = 0;
            TMIN[i] = kNone32;
            ST[i] = 0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            const uint32_t i = tid + k * kWG;
            if (i < n) {
                const uint32_t rr = root[k];
                const Ev& e = ev[k];
                atomicAdd(&W[rr], e.tot);
                atomicAdd(&SX[rr], e.tot * e.x);
                atomicAdd(&SY[rr], e.tot * e.y);
                atomicAdd(&CNT[rr], 1u);
                atomicMin(&TMIN[rr], e.t);
                atomicAdd(&ST[rr], (unsigned long long)time_term(a, e.tot, e.t));
            }
        }
        __syncthreads();
        // hits without any ToT: plain means (the weighted sums are all zero)
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            const uint32_t i = tid + k * kWG;
            if (i < n && W[root[k]] == 0) {
                const uint32_t rr = root[k];
                atomicAdd(&SX[rr], ev[k].x);
                atomicAdd(&SY[rr], ev[k].y);
                atomicAdd(&ST[rr], (unsigned long long)time_term1(a, ev[k].tot, ev[k].t));
            }
        }
        __syncthreads();
        uint32_t rank[kK];
        uint32_t running = 0;
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            const uint32_t i = tid + k * kWG;
            uint32_t tot;
            const bool is_root = i < n && root[k] == i;
            rank[k] = running + wg_flag_scan<kWG>(is_root, scan_tmp, &tot);
            running += tot;
        }
        if (tid < 64) {
            const uint64_t p = seg_lookback(a, ticket, running);
            if (tid == 0) {
                bc[1] = p;
                if (running) atomicAdd(&a.res->n_hits, (unsigned long long)running);
            }
        }
        __syncthreads();
        const uint64_t out0 = bc[1];
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            const uint32_t i = tid + k * kWG;
            if (i < n && root[k] == i)
                write_hit(a, out0 + rank[k], ev[k].g, W[i], CNT[i], SX[i], SY[i], ST[i], TMIN[i],
                          gidx_of(a, e0 + i));
        }
    }
}

// ------------------------------------------------------ global-memory segment
template <bool kEvent>
__device__ void seg_big(const ClusterArgs& a, uint8_t* lds, uint32_t* scan_tmp, uint64_t* bc,
                        uint32_t g_lo, uint32_t ng, uint64_t e0, uint32_t n, uint64_t ticket) {
    uint32_t* img = (uint32_t*)lds;  // u32[kH], all-ones = empty
    uint32_t* par = a.g_parent + e0;
    uint32_t* chn = a.g_chain + e0;
    uint32_t* nxt = a.g_next + e0;
    uint32_t* tt = a.g_t + e0;
    uint32_t* sl = a.g_sl + e0;
    uint32_t* xy = a.g_xy + e0;
    const int tid = threadIdx.x;
    const int r = (int)a.dxy;
    const uint32_t dt = a.dt;
    unsigned long long* err = &a.res->err;
    if (tid == 0) atomicAdd(&a.res->big_segments, 1ull);
    {
        uint4* v = (uint4*)img;
        for (int i = tid; i < kH * 4 / 16; i += kWG) v[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
    }
    for (uint32_t i = tid; i < n; i += kWG) {
        Ev e;
        load_event<kEvent>(a, e0 + i, nullptr, 0, ng, false, g_lo, e, err);
        par[i] = i;
        chn[i] = kNone32;
        tt[i] = e.t;
        sl[i] = e.g;
        xy[i] = e.x | (e.y << 8) | (e.tot << 16);
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint32_t v = xy[i];
        img[slot_of(v & 255u, (v >> 8) & 255u)] = i;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint32_t v = xy[i];
        const uint32_t w = img[slot_of(v & 255u, (v >> 8) & 255u)];
        if (w != i) nxt[i] = atomicExch(&chn[w], i);
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint32_t v = xy[i];
        const int x = (int)(v & 255u), y = (int)((v >> 8) & 255u);
        for (int dy = 0; dy <= r; ++dy) {
            const int ny = y + dy;
            if (ny > 255) break;
            for (int dx = (dy == 0 ? 0 : -r); dx <= r; ++dx) {
                const int nx = x + dx;
                if (nx < 0 || nx > 255) continue;
                visit_slot(img, chn, nxt, tt, sl, xy, par, i, x, y, tt[i], sl[i], nx, ny,
                           dx == 0 && dy == 0, r, dt, n, kNone32, err);
            }
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kWG) chn[i] = uf_find(par, i, n, err);  // root
    __syncthreads();
    if constexpr (kEvent) {
        uint32_t nroot = 0;
        for (uint32_t i = tid; i < n; i += kWG) {
            const uint32_t rt = chn[i];
            a.labels[orig_of(a, e0 + i)] = (uint32_t)orig_of(a, e0 + rt);
            nroot += rt == i;
        }
        for (int d = 32; d > 0; d >>= 1) nroot += __shfl_xor(nroot, d, 64);
        if (__lane_id() == 0 && nroot) atomicAdd(&a.res->n_hits, (unsigned long long)nroot);
    } else {
        unsigned long long* acc = (unsigned long long*)a.g_acc + 6 * e0;
        for (uint32_t i = tid; i < n; i += kWG) {
            acc[6 * i + 0] = 0;      // W
            acc[6 * i + 1] = 0;      // count
            acc[6 * i + 2] = 0;      // Sx
            acc[6 * i + 3] = 0;      // Sy
            acc[6 * i + 4] = 0;      // St
            acc[6 * i + 5] = ~0ull;  // min t
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kWG) {
            const uint32_t rt = chn[i], v = xy[i], t = tt[i];
            const uint32_t x = v & 255u, y = (v >> 8) & 255u, tot = v >> 16;
            unsigned long long* q = acc + 6 * rt;
            atomicAdd(q + 0, (unsigned long long)tot);
            atomicAdd(q + 1, 1ull);
            atomicAdd(q + 2, (unsigned long long)(tot * x));
            atomicAdd(q + 3, (unsigned long long)(tot * y));
            atomicAdd(q + 4, (unsigned long long)time_term(a, tot, t));
            atomicMin(q + 5, (unsigned long long)t);
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kWG) {
            unsigned long long* q = acc + 6 * chn[i];
            if (q[0] == 0) {
                const uint32_t v = xy[i];
                atomicAdd(q + 2, (unsigned long long)(v & 255u));
                atomicAdd(q + 3, (unsigned long long)((v >> 8) & 255u));
                atomicAdd(q + 4, (unsigned long long)time_term1(a, v >> 16, tt[i]));
            }
        }
        __syncthreads();
        // ranks of the roots in position order, one workgroup-wide round at a time
        uint32_t running = 0;
        const uint32_t rounds = (n + kWG - 1) / kWG;
        for (uint32_t rd = 0; rd < rounds; ++rd) {
            const uint32_t i = rd * kWG + tid;
            uint32_t tot;
            const bool is_root = i < n && chn[i] == i;
            const uint32_t rk = running + wg_flag_scan<kWG>(is_root, scan_tmp, &tot);
            if (is_root) par[i] = rk;  // parents are no longer needed: keep the rank
            running += tot;
        }
        if (tid < 64) {
            const uint64_t p = seg_lookback(a, ticket, running);
            if (tid == 0) {
                bc[1] = p;
                if (running) atomicAdd(&a.res->n_hits, (unsigned long long)running);
            }
        }
        __syncthreads();
        const uint64_t out0 = bc[1];
        for (uint32_t i = tid; i < n; i += kWG) {
            if (chn[i] == i) {
                const unsigned long long* q = acc + 6 * i;
                write_hit(a, out0 + par[i], sl[i], q[0], q[1], q[2], q[3], q[4], (uint32_t)q[5],
                          gidx_of(a, e0 + i));
            }
        }
    }
}

// Segment table: seg_lo[k] = first group whose first event is at or after
// k q, for k = 0..n_seg (n_seg = ceil(N / q)).  One thread per group g = 0..G
// fills the k in (grp_off[g-1] / q, grp_off[g] / q]; g = G closes at n_seg.
__global__ void k_seg_table(const uint32_t* __restrict__ grp_off, const unsigned long long* n_grp_dev,
                            const unsigned long long* n_ev_dev, const unsigned long long* skip,
                            uint32_t q, uint32_t* seg_lo) {
    if (skip && *skip) return;
    const uint64_t G = *n_grp_dev, N = *n_ev_dev;
    const uint64_t n_seg = (N + q - 1) / q;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= G;
         g += (uint64_t)gridDim.x * blockDim.x) {
        // offsets never exceed N in a valid table; the clamps keep every
        // write inside seg_lo[0..n_seg] whatever the table holds
        const int64_t k_prev = g == 0 ? -1 : (int64_t)min<uint64_t>(grp_off[g - 1] / q, n_seg);
        const int64_t k_hi = g == G ? (int64_t)n_seg : (int64_t)min<uint64_t>(grp_off[g] / q, n_seg);
        for (int64_t k = k_prev + 1; k <= k_hi; ++k) seg_lo[k] = (uint32_t)g;
    }
}

void launch_seg_table(const uint32_t* grp_off, const unsigned long long* n_grp_dev,
                      const unsigned long long* n_ev_dev, const unsigned long long* skip,
                      uint32_t q, uint64_t max_groups, uint32_t* seg_lo, hipStream_t s) {
    uint64_t blocks = (max_groups + 1 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_seg_table, dim3((unsigned)blocks), dim3(256), 0, s, grp_off, n_grp_dev,
                       n_ev_dev, skip, q, seg_lo);
}

// One workgroup per segment.  The grid covers the largest possible number of
// segments; workgroups whose ticket is beyond the actual count return at once.
template <bool kEvent>
__global__ __launch_bounds__(kWG, 2) void k_cluster(ClusterArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsMain];
    __shared__ uint32_t scan_tmp[kWG / 64 + 1];
    __shared__ uint64_t bc[8];
    __shared__ uint32_t goff[kWG + 1];
    const int tid = threadIdx.x;
    if (tid == 0) bc[0] = atomicAdd(&a.res->seg_ticket, 1ull);
    __syncthreads();
    const uint32_t k = __builtin_amdgcn_readfirstlane((uint32_t)bc[0]);
    const uint64_t N = (a.skip && *a.skip) ? 0 : *a.n_ev_dev;
    const uint64_t n_seg = (N + a.q - 1) / a.q;
    if (k >= n_seg) return;
    // groups whose first event lies in [k q, (k+1) q)
    const uint32_t g_lo = a.seg_lo[k], g_hi = a.seg_lo[k + 1];
    const uint64_t e0 = a.grp_off[g_lo], e1 = a.grp_off[g_hi];
    if (g_hi < g_lo || e1 < e0 || e1 > N) {
        if (tid == 0) {
            atomicOr(&a.res->err, (unsigned long long)kErrInternal);
            if (!kEvent) lb_publish(a.lb_status, k, kLbAggregate, 0);
        }
        return;
    }
    const uint32_t n = (uint32_t)(e1 - e0);
    const uint32_t ng = g_hi - g_lo;
    if (n == 0) {
        if constexpr (!kEvent) {
            if (tid == 0) lb_publish(a.lb_status, k, k == 0 ? kLbInclusive : kLbAggregate, 0);
        }
        return;
    }
    if (n <= (uint32_t)kCap) {
        const bool goff_lds = ng <= (uint32_t)kWG;
        if (goff_lds) {
            for (uint32_t i = tid; i <= ng; i += kWG) goff[i] = a.grp_off[g_lo + i];
        }
        __syncthreads();
        seg_small<kEvent>(a, lds, scan_tmp, bc, goff, goff_lds, g_lo, ng, e0, n, k);
    } else {
        seg_big<kEvent>(a, lds, scan_tmp, bc, g_lo, ng, e0, n, k);
    }
    if (tid == 0) atomicMax(&a.res->max_segment, (unsigned long long)n);
}

uint64_t cluster_grid(uint64_t max_events, uint32_t q) { return max_events / q + 2; }

void launch_cluster(const ClusterArgs& a, bool event_mode, uint64_t grid, hipStream_t s) {
    if (grid == 0) return;
    if (event_mode)
        hipLaunchKernelGGL(k_cluster<true>, dim3((unsigned)grid), dim3(kWG), 0, s, a);
    else
        hipLaunchKernelGGL(k_cluster<false>, dim3((unsigned)grid), dim3(kWG), 0, s, a);
}

int cluster_capacity() { return kCap; }

}  // namespace tpx
