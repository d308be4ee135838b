// Connectivity clustering and ToT-weighted centroids (Sec. V: Neighborhoods,
// Eqs. 3-5, closed transitively; Centroiding, Eqs. 8-9).
//
// Events arrive grouped by shot.  Groups are packed into segments of about
// `q` events (the groups whose first event lies in [k q, (k+1) q)); the
// segment table comes from k_seg_table.
//
// k_cluster, one workgroup per segment, finds the components of the
// neighbourhood graph (same shot, |dx|, |dy| <= r, |dt| <= r_t: the edges of
// the paper's Hadamard adjacency A) in four steps over LDS:
//   1. every event is dropped into a hashed 256x64 image of its pixel address;
//      events sharing an image slot are chained behind the slot owner;
//   2. every event points at the smallest event among itself and its
//      neighbours (a plain store: no atomics), which makes a forest whose
//      roots are local minima;
//   3. after path compression, each edge of the forward half-neighbourhood
//      whose ends lie in different trees is united (lock-free union-find that
//      hooks the larger root under the smaller); most edges are already
//      inside one tree;
//   4. a final find gives each event its root = the smallest event position
//      of its component = its label.
// In event mode (tpx_cluster) the kernel writes labels.  In stream mode it
// writes, for every event, the rank of its component within the segment
// (components ordered by label) and the segment's component count; after a
// prefix sum over segments, k_seg_centroid accumulates exact integer moments
// per component and writes one hit per component at its final position, so no
// segment ever waits for another.  Segments larger than the LDS capacity take
// the same steps with their per-event arrays in global memory.
#include "tpx_decode_dev.h"
#include "tpx_util_dev.h"

namespace tpx {

constexpr int kCap = 2048;             // events per segment held in LDS
constexpr int kWG = 512;               // threads per workgroup (k_cluster)
constexpr int kH = 16384;              // image slots: (y & 63) << 8 | x
constexpr uint32_t kNone32 = 0xFFFFFFFFu;
constexpr uint32_t kNone16 = 0xFFFFu;

// LDS byte layout of k_cluster's small-segment path
constexpr int kOffImg = 0;             // u16[kH] slot owner
constexpr int kOffPar = 32768;         // u32[kCap] union-find parent
constexpr int kOffEv = 40960;          // u64[kCap] x | y << 8 | group start << 16 | t << 32
constexpr int kOffChn = 57344;         // u32[kCap] first chained event of a slot owner
constexpr int kOffNxt = 65536;         // u16[kCap] next chained event
constexpr int kOffMsk = 69632;         // u32[kCap] neighbour mask (3x3 box)
constexpr int kLdsMain = 77824;
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

// group (shot) of sorted position p: last g in [lo, hi) with off[g] <= p
template <typename P>
__device__ inline uint32_t group_of(P off, uint32_t lo, uint32_t hi, uint32_t p) {
    while (hi - lo > 1) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (off[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

// Segment k: groups [g_lo, g_hi), events [e0, e0 + n).  False (and the
// internal-error flag) when the tables are inconsistent.
struct Seg {
    uint32_t g_lo, g_hi, n;
    uint64_t e0;
};
__device__ inline bool seg_bounds(const ClusterArgs& a, uint32_t k, uint64_t N, Seg& s) {
    s.g_lo = a.seg_lo[k];
    s.g_hi = a.seg_lo[k + 1];
    s.e0 = a.grp_off[s.g_lo];
    const uint64_t e1 = a.grp_off[s.g_hi];
    if (s.g_hi < s.g_lo || e1 < s.e0 || e1 > N) {
        if (threadIdx.x == 0) atomicOr(&a.res->err, (unsigned long long)kErrInternal);
        return false;
    }
    s.n = (uint32_t)(e1 - s.e0);
    return true;
}

__device__ inline uint64_t n_events(const ClusterArgs& a) {
    return (a.skip && *a.skip) ? 0 : *a.n_ev_dev;
}

// Pixel address, time and the first position of its group (relative to the
// segment start), for the event at sorted position p of group g.
struct Ev {
    uint32_t x, y, t, gs;
};

template <bool kEvent>
__device__ inline Ev load_event(const ClusterArgs& a, uint64_t p, uint32_t g, uint64_t e0,
                                unsigned long long* err) {
    Ev e;
    const uint64_t first = a.grp_off[g];
    e.gs = (uint32_t)(first - e0);
    if constexpr (!kEvent) {
        const uint64_t pk = a.ev[p];
        e.x = ev_x(pk);
        e.y = ev_y(pk);
        e.t = ev_t(pk);
    } else {
        const uint64_t o = a.perm ? a.perm[p] : p;
        e.x = a.soa.x[o];
        e.y = a.soa.y[o];
        const uint64_t of = a.perm ? a.perm[first] : first;
        const uint64_t d = a.soa.toa[o] - a.soa.toa[of] + (1ull << 31);
        if (e.x > 255u || e.y > 255u || d >= (1ull << 32)) {
            atomicOr(err, (unsigned long long)kErrInput);
            e.x &= 255u;
            e.y &= 255u;
        }
        e.t = (uint32_t)d;
    }
    return e;
}

__device__ inline uint64_t pack_lds(const Ev& e) {
    return (uint64_t)e.x | ((uint64_t)e.y << 8) | ((uint64_t)e.gs << 16) | ((uint64_t)e.t << 32);
}

// global event index of sorted position p (stream path)
__device__ inline uint64_t gidx_of(const ClusterArgs& a, uint64_t p) {
    const uint64_t o = a.perm ? a.perm[p] : p;
    return o < a.n_carry ? a.carry_gidx[o] : a.ev_base + (o - a.n_carry);
}

__device__ inline uint64_t orig_of(const ClusterArgs& a, uint64_t p) {
    return a.perm ? a.perm[p] : p;
}

// Calls f(j) for every event j in image slot (nx, ny): the owner, then its
// chain.  Returns false when a chain is longer than the segment.
template <typename F>
__device__ inline bool slot_events(const uint16_t* img, const uint32_t* chn, const uint16_t* nxt,
                                   int nx, int ny, uint32_t n, F&& f) {
    const uint32_t w = img[slot_of((uint32_t)nx, (uint32_t)ny)];
    if (w == kNone16) return true;
    f(w);
    uint32_t j = chn[w];
    uint32_t steps = 0;
    while (j != kNone32) {
        f(j);
        if (++steps > n) return false;
        const uint32_t nn = nxt[j];
        j = nn == kNone16 ? kNone32 : nn;
    }
    return true;
}

// Calls f(j, fwd) for every event j != i in the image slots of the
// (2r+1)^2 box around (x, y); fwd marks the forward half (later rows, later
// columns of the same row, and smaller positions in the event's own slot),
// which holds every undirected edge exactly once.  R > 0 fixes the radius at
// compile time (unrolled); R == 0 takes it from r_rt.
template <int R, typename F>
__device__ inline bool box_events(const uint16_t* img, const uint32_t* chn, const uint16_t* nxt,
                                  uint32_t i, int x, int y, int r_rt, uint32_t n, F&& f) {
    bool ok = true;
    auto one = [&](int dx, int dy) {
        const int nx = x + dx, ny = y + dy;
        if (nx < 0 || nx > 255 || ny < 0 || ny > 255) return;
        const bool fwd_slot = dy > 0 || (dy == 0 && dx > 0);
        const bool own = dx == 0 && dy == 0;
        ok &= slot_events(img, chn, nxt, nx, ny, n, [&](uint32_t j) {
            if (j != i) f(j, fwd_slot || (own && j < i));
        });
    };
    if constexpr (R > 0) {
#pragma unroll
        for (int dy = -R; dy <= R; ++dy)
#pragma unroll
            for (int dx = -R; dx <= R; ++dx) one(dx, dy);
    } else {
        for (int dy = -r_rt; dy <= r_rt; ++dy)
            for (int dx = -r_rt; dx <= r_rt; ++dx) one(dx, dy);
    }
    return ok;
}

// Edge test for a candidate taken from image slot (x + dx, (y + dy) & 63): x
// matches by construction, y up to multiples of 64.
__device__ inline bool is_edge_slot(uint64_t me, uint64_t o, int dy, uint32_t dt) {
    const uint32_t ya = (uint32_t)(me >> 8) & 255u, yb = (uint32_t)(o >> 8) & 255u;
    return ((me ^ o) & 0xFFFF0000ull) == 0 &&                           // same group
           absdiff((uint32_t)(me >> 32), (uint32_t)(o >> 32)) <= dt &&  // |dt|
           yb == ya + (uint32_t)dy;
}

__device__ inline bool is_edge(uint64_t me, uint64_t o, int r, uint32_t dt) {
    const uint32_t ya = (uint32_t)(me >> 8) & 255u, yb = (uint32_t)(o >> 8) & 255u;
    const uint32_t xa = (uint32_t)me & 255u, xb = (uint32_t)o & 255u;
    return ((me ^ o) & 0xFFFF0000ull) == 0 &&                           // same group
           absdiff((uint32_t)(me >> 32), (uint32_t)(o >> 32)) <= dt &&  // |dt|
           absdiff(ya, yb) <= (uint32_t)r && absdiff(xa, xb) <= (uint32_t)r;
}

// ---------------------------------------------------- 3x3 box (r = 1)
// Slot s of the box is (x + s % 3 - 1, y + s / 3 - 1).  Every event sees the
// owner of each slot and the first event chained behind it (18 candidates).
// Mask bit s: the owner of slot s is a neighbour; bit 9 + s: its first chained
// event is.  An event deeper in a chain (kDeep) is invisible to the others, so
// it records its edges to the 18 candidates whatever their positions and
// walks the rest of the chains itself; otherwise only candidates with smaller
// positions are recorded, so that every edge is recorded once.
constexpr uint32_t kDeep = 1u << 18;
constexpr uint32_t kMaxRounds = 64;

__device__ inline bool box3_slot(int x, int y, int s, uint32_t* slot) {
    const int nx = x + s % 3 - 1, ny = y + s / 3 - 1;
    *slot = slot_of((uint32_t)nx, (uint32_t)ny);
    return nx >= 0 && nx <= 255 && ny >= 0 && ny <= 255;
}

// Candidate 0..17 of event v: owners, then first chained events (kNone32 if
// none).
__device__ inline void box3_cands(const uint16_t* img, const uint32_t* chn, uint64_t v,
                                  uint32_t* c) {
    const int x = (int)(v & 255u), y = (int)((v >> 8) & 255u);
#pragma unroll
    for (int s = 0; s < 9; ++s) {
        uint32_t slot;
        const bool in = box3_slot(x, y, s, &slot);
        const uint32_t w = in ? (uint32_t)img[slot] : kNone16;
        c[s] = w == kNone16 ? kNone32 : w;
    }
#pragma unroll
    for (int s = 0; s < 9; ++s) c[9 + s] = c[s] == kNone32 ? kNone32 : chn[c[s]];
}

// Mask of event i (see above) and its smallest recorded neighbour (or i).
__device__ inline uint32_t box3_visit(const uint16_t* img, const uint32_t* chn,
                                      const uint16_t* nxt, const uint64_t* evs, uint32_t i,
                                      uint32_t dt, uint32_t* m_out) {
    const uint64_t v = evs[i];
    uint32_t c[18];
    box3_cands(img, chn, v, c);
    uint64_t e[18];
#pragma unroll
    for (int s = 0; s < 18; ++s) e[s] = evs[c[s] == kNone32 ? i : c[s]];
    // i is deep when it is neither the owner nor the first chained event of
    // its own slot
    const bool deep = c[4] != i && c[13] != i;
    uint32_t m = i, mask = deep ? kDeep : 0u;
#pragma unroll
    for (int s = 0; s < 18; ++s) {
        const uint32_t j = c[s];
        const bool ed = j != kNone32 && j != i && (deep || j < i) &&
                        is_edge_slot(v, e[s], (s % 9) / 3 - 1, dt);
        mask |= ed ? (1u << s) : 0u;
        m = (ed && j < m) ? j : m;
    }
    *m_out = m;
    return mask;
}

// Calls f(q) for every event q != i chained at depth two or more in the box
// of v with an edge to v.  False when a chain is longer than the segment.
template <typename F>
__device__ inline bool box3_deep_edges(const uint16_t* img, const uint32_t* chn,
                                       const uint16_t* nxt, const uint64_t* evs, uint32_t i,
                                       uint64_t v, uint32_t dt, uint32_t n, F&& f) {
    uint32_t c[18];
    box3_cands(img, chn, v, c);
    bool ok = true;
    for (int s = 9; s < 18; ++s) {
        if (c[s] == kNone32) continue;
        const uint32_t first = nxt[c[s]];
        uint32_t q = first == kNone16 ? kNone32 : first, steps = 0;
        while (q != kNone32) {
            if (q != i && is_edge(v, evs[q], 1, dt)) f(q);
            if (++steps > n) {
                ok = false;
                break;
            }
            const uint32_t nn = nxt[q];
            q = nn == kNone16 ? kNone32 : nn;
        }
    }
    return ok;
}

// Hooks the larger of two distinct tree roots under the smaller if it is
// still a root: trees only ever merge, so two events once seen in one tree
// stay in one tree.  False when the root was taken by another hook first (the
// edge is then seen again in the next round).
__device__ inline bool hook(uint32_t* par, uint32_t ra, uint32_t rb) {
    const uint32_t hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
    uint32_t expect = hi;
    return __hip_atomic_compare_exchange_strong(par + hi, &expect, lo, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Points every event at its root (pointer jumping; concurrent readers see an
// old parent or a root, both ancestors).
__device__ inline void compress_all(uint32_t* par, uint32_t n, int tid, int nthreads) {
    for (uint32_t i = tid; i < n; i += nthreads) {
        uint32_t p = ald(par + i), steps = 0;
        for (uint32_t nx; p != (nx = ald(par + p)) && ++steps <= n;) p = nx;
        ast(par + i, p);
    }
}

// ------------------------------------------------------------ LDS segment
// Every phase walks the events i = tid + q kWG, q < kK; per-event state lives
// in LDS between phases.
template <bool kEvent, int R>
__device__ void seg_small(const ClusterArgs& a, uint8_t* lds, uint32_t* scan_tmp,
                          const uint32_t* goff, bool goff_lds, const Seg& sg, uint32_t k) {
    uint16_t* img = (uint16_t*)(lds + kOffImg);
    uint32_t* par = (uint32_t*)(lds + kOffPar);
    uint64_t* evs = (uint64_t*)(lds + kOffEv);
    uint32_t* chn = (uint32_t*)(lds + kOffChn);
    uint16_t* nxt = (uint16_t*)(lds + kOffNxt);
    uint32_t* msk = (uint32_t*)(lds + kOffMsk);
    const int tid = threadIdx.x;
    const int r = (int)a.dxy;
    const uint32_t dt = a.dt, n = sg.n;
    const uint64_t e0 = sg.e0;
    unsigned long long* err = &a.res->err;

    {
        uint4* v = (uint4*)img;
        for (int i = tid; i < kH * 2 / 16; i += kWG) v[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
    }
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint32_t p = (uint32_t)(e0 + i);
        const uint32_t g = goff_lds ? sg.g_lo + group_of(goff, 0, sg.g_hi - sg.g_lo, p)
                                    : group_of(a.grp_off, sg.g_lo, sg.g_hi, p);
        evs[i] = pack_lds(load_event<kEvent>(a, e0 + i, g, e0, err));
        chn[i] = kNone32;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint64_t v = evs[i];
        img[slot_of((uint32_t)v & 255u, (uint32_t)(v >> 8) & 255u)] = (uint16_t)i;
    }
    __syncthreads();
    // events that lost the race for their slot chain behind the owner
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint64_t v = evs[i];
        const uint32_t w = img[slot_of((uint32_t)v & 255u, (uint32_t)(v >> 8) & 255u)];
        if (w != i) {
            const uint32_t old = atomicExch(&chn[w], i);
            nxt[i] = (uint16_t)(old == kNone32 ? kNone16 : old);
        }
    }
    __syncthreads();
    bool ok = true;
    if constexpr (R == 1) {
        // every event points at its smallest recorded neighbour (or itself):
        // a forest whose roots are local minima
        for (uint32_t i = tid; i < n; i += kWG) {
            uint32_t m;
            const uint32_t mask = box3_visit(img, chn, nxt, evs, i, dt, &m);
            if (mask & kDeep)
                ok &= box3_deep_edges(img, chn, nxt, evs, i, evs[i], dt, n,
                                      [&](uint32_t q) { m = q < m ? q : m; });
            par[i] = m;
            msk[i] = mask;
        }
        __syncthreads();
        compress_all(par, n, tid, kWG);
        __syncthreads();
        // rounds of root hooks over the recorded edges, then pointer jumping;
        // an edge whose ends share a tree, or whose hook took, is dropped for
        // good (trees never split); a round in which every hook took ends it
        for (uint32_t round = 0;; ++round) {
            bool changed = false;  // some edge still to be seen again
            for (uint32_t i = tid; i < n; i += kWG) {
                const uint32_t mask = msk[i];
                if (!mask) continue;
                const uint64_t v = evs[i];
                const int x = (int)(v & 255u), y = (int)((v >> 8) & 255u);
                const uint32_t ri = ald(par + i);
                uint32_t keep = mask & kDeep;
                // the recorded candidates only, one set bit at a time
                for (uint32_t bits = mask & (kDeep - 1); bits; bits &= bits - 1) {
                    const int s = __builtin_ctz(bits);
                    uint32_t slot;
                    box3_slot(x, y, s % 9, &slot);
                    const uint32_t w = img[slot];
                    const uint32_t j = s < 9 ? w : chn[w];
                    const uint32_t rj = ald(par + j);
                    if (rj != ri && !hook(par, ri, rj)) {
                        keep |= 1u << s;
                        changed = true;
                    }
                }
                if (mask & kDeep)
                    ok &= box3_deep_edges(img, chn, nxt, evs, i, v, dt, n, [&](uint32_t q) {
                        const uint32_t ra = ald(par + i), rq = ald(par + q);
                        if (q < i && ra != rq && !hook(par, ra, rq)) changed = true;
                    });
                if (keep != mask) msk[i] = keep;
            }
            __syncthreads();
            compress_all(par, n, tid, kWG);
            if (!__syncthreads_or(changed)) break;
            if (round >= kMaxRounds) {  // far more rounds than any forest needs
                if (tid == 0) atomicOr(err, (unsigned long long)kErrLoopUnite);
                break;
            }
        }
    } else {
        // every event points at the smallest of itself and its neighbours
        for (uint32_t i = tid; i < n; i += kWG) {
            uint32_t m = i;
            const uint64_t v = evs[i];
            ok &= box_events<R>(img, chn, nxt, i, (int)(v & 255u), (int)((v >> 8) & 255u), r, n,
                                [&](uint32_t j, bool) {
                                    if (j < m && is_edge(v, evs[j], r, dt)) m = j;
                                });
            par[i] = m;
        }
        __syncthreads();
        compress_all(par, n, tid, kWG);
        __syncthreads();
        // edges between different trees
        for (uint32_t i = tid; i < n; i += kWG) {
            const uint64_t v = evs[i];
            ok &= box_events<R>(img, chn, nxt, i, (int)(v & 255u), (int)((v >> 8) & 255u), r, n,
                                [&](uint32_t j, bool fwd) {
                                    if (fwd && ald(par + j) != ald(par + i) &&
                                        is_edge(v, evs[j], r, dt))
                                        uf_unite(par, i, j, n, err);
                                });
        }
        __syncthreads();
        // final roots, stored as parents
        for (uint32_t i = tid; i < n; i += kWG) ast(par + i, uf_find(par, i, n, err));
    }
    if (!ok) atomicOr(err, (unsigned long long)kErrLoopChain);
    __syncthreads();

    if constexpr (kEvent) {
        uint32_t nroot = 0;
        for (uint32_t i = tid; i < n; i += kWG) {
            const uint32_t rt = par[i];
            a.labels[orig_of(a, e0 + i)] = (uint32_t)orig_of(a, e0 + rt);
            nroot += rt == i;
        }
        for (int d = 32; d > 0; d >>= 1) nroot += __shfl_xor(nroot, d, 64);
        if (__lane_id() == 0 && nroot) atomicAdd(&a.res->n_hits, (unsigned long long)nroot);
    } else {
        // rank of every component (in label order) within the segment, kept
        // at the root's chain slot (chains are no longer needed)
        uint32_t running = 0;
        const uint32_t rounds = (n + kWG - 1) / kWG;
        for (uint32_t rd = 0; rd < rounds; ++rd) {
            const uint32_t i = rd * kWG + tid;
            uint32_t tot;
            const bool is_root = i < n && par[i] == i;
            const uint32_t rk = running + wg_flag_scan<kWG>(is_root, scan_tmp, &tot);
            if (is_root) chn[i] = rk;
            running += tot;
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kWG) a.rank[e0 + i] = chn[par[i]];
        if (tid == 0) a.seg_cnt[k] = running;
    }
}

// ------------------------------------------------------ global-memory segment
template <bool kEvent>
__device__ void seg_big(const ClusterArgs& a, uint8_t* lds, uint32_t* scan_tmp, const Seg& sg,
                        uint32_t k) {
    uint32_t* img = (uint32_t*)lds;  // u32[kH], all-ones = empty
    const uint64_t e0 = sg.e0;
    const uint32_t n = sg.n;
    uint32_t* par = a.g_parent + e0;
    uint32_t* chn = a.g_chain + e0;
    uint32_t* nxt = a.g_next + e0;
    uint32_t* tt = a.g_t + e0;
    uint32_t* gs = a.g_sl + e0;
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
        const uint32_t g = group_of(a.grp_off, sg.g_lo, sg.g_hi, (uint32_t)(e0 + i));
        const Ev e = load_event<kEvent>(a, e0 + i, g, e0, err);
        par[i] = i;
        chn[i] = kNone32;
        tt[i] = e.t;
        gs[i] = e.gs;
        xy[i] = e.x | (e.y << 8);
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
        const uint32_t t = tt[i], g = gs[i];
        for (int dy = 0; dy <= r; ++dy) {
            const int ny = y + dy;
            if (ny > 255) break;
            for (int dx = (dy == 0 ? 0 : -r); dx <= r; ++dx) {
                const int nx = x + dx;
                if (nx < 0 || nx > 255) continue;
                const bool own = dx == 0 && dy == 0;
                const uint32_t w = img[slot_of((uint32_t)nx, (uint32_t)ny)];
                uint32_t j = w;
                uint32_t steps = 0;
                while (j != kNone32) {
                    if (j != i && (!own || j < i)) {
                        const uint32_t vj = xy[j];
                        if (gs[j] == g && absdiff(tt[j], t) <= dt &&
                            abs((int)(vj & 255u) - x) <= r && abs((int)((vj >> 8) & 255u) - y) <= r)
                            uf_unite(par, i, j, n, err);
                    }
                    if (++steps > n) {
                        atomicOr(err, (unsigned long long)kErrLoopChain);
                        break;
                    }
                    j = (j == w) ? chn[j] : nxt[j];
                }
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
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kWG) a.rank[e0 + i] = par[chn[i]];
        if (tid == 0) a.seg_cnt[k] = running;
    }
}

// Segment table: seg_lo[k] = first group whose first event is at or after
// k q, for k = 0..n_seg (n_seg = ceil(N / q)).  One thread per group g = 0..G
// fills the k in (grp_off[g-1] / q, grp_off[g] / q]; g = G closes at n_seg.
__device__ __forceinline__ void seg_table_range(const uint32_t* __restrict__ grp_off,
                                const unsigned long long* n_grp_dev,
                                const unsigned long long* n_ev_dev, const unsigned long long* skip,
                                uint32_t q, uint32_t* seg_lo, DevResults* res, uint64_t first,
                                uint64_t stride) {
    const bool sk = skip && *skip;
    const uint64_t G = *n_grp_dev, N = sk ? 0 : *n_ev_dev;
    const uint64_t n_seg = (N + q - 1) / q;
    if (first == 0) res->n_seg = n_seg;
    if (sk) return;
    for (uint64_t g = first; g <= G; g += stride) {
        // offsets never exceed N in a valid table; the clamps keep every
        // write inside seg_lo[0..n_seg] whatever the table holds
        const int64_t k_prev = g == 0 ? -1 : (int64_t)min<uint64_t>(grp_off[g - 1] / q, n_seg);
        const int64_t k_hi = g == G ? (int64_t)n_seg : (int64_t)min<uint64_t>(grp_off[g] / q, n_seg);
        for (int64_t k = k_prev + 1; k <= k_hi; ++k) seg_lo[k] = (uint32_t)g;
    }
}
__global__ void k_seg_table(const uint32_t* __restrict__ grp_off, const unsigned long long* n_grp_dev,
                            const unsigned long long* n_ev_dev, const unsigned long long* skip,
                            uint32_t q, uint32_t* seg_lo, DevResults* res) {
    seg_table_range(grp_off, n_grp_dev, n_ev_dev, skip, q, seg_lo, res,
                    (uint64_t)blockIdx.x * blockDim.x + threadIdx.x,
                    (uint64_t)gridDim.x * blockDim.x);
}

void launch_seg_table(const uint32_t* grp_off, const unsigned long long* n_grp_dev,
                      const unsigned long long* n_ev_dev, const unsigned long long* skip,
                      uint32_t q, uint64_t max_groups, uint32_t* seg_lo, DevResults* res,
                      hipStream_t s) {
    uint64_t blocks = (max_groups + 1 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_seg_table, dim3((unsigned)blocks), dim3(256), 0, s, grp_off, n_grp_dev,
                       n_ev_dev, skip, q, seg_lo, res);
}

// One workgroup per segment; the grid covers the largest possible number of
// segments and workgroups beyond the actual count return at once.
template <bool kEvent, int R>
__global__ __launch_bounds__(kWG, 2) void k_cluster(ClusterArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsMain];
    __shared__ uint32_t scan_tmp[kWG / 64 + 1];
    __shared__ uint32_t goff[kWG + 1];
    const int tid = threadIdx.x;
    const uint32_t k = blockIdx.x;
    const uint64_t N = n_events(a);
    const uint64_t n_seg = (N + a.q - 1) / a.q;
    if (k >= n_seg) return;
    Seg sg;
    if (!seg_bounds(a, k, N, sg)) return;
    if (sg.n == 0) {
        if (!kEvent && tid == 0) a.seg_cnt[k] = 0;
        return;
    }
    const uint32_t ng = sg.g_hi - sg.g_lo;
    if (sg.n <= (uint32_t)kCap) {
        const bool goff_lds = ng <= (uint32_t)kWG;
        if (goff_lds) {
            for (uint32_t i = tid; i <= ng; i += kWG) goff[i] = a.grp_off[sg.g_lo + i];
        }
        __syncthreads();
        seg_small<kEvent, R>(a, lds, scan_tmp, goff, goff_lds, sg, k);
    } else {
        seg_big<kEvent>(a, lds, scan_tmp, sg, k);
    }
}

uint64_t cluster_grid(uint64_t max_events, uint32_t q) { return max_events / q + 2; }

void launch_cluster(const ClusterArgs& a, bool event_mode, uint64_t grid, hipStream_t s) {
    if (grid == 0) return;
    const bool r1 = a.dxy == 1;
    if (event_mode) {
        if (r1) hipLaunchKernelGGL((k_cluster<true, 1>), dim3((unsigned)grid), dim3(kWG), 0, s, a);
        else hipLaunchKernelGGL((k_cluster<true, 0>), dim3((unsigned)grid), dim3(kWG), 0, s, a);
    } else {
        if (r1) hipLaunchKernelGGL((k_cluster<false, 1>), dim3((unsigned)grid), dim3(kWG), 0, s, a);
        else hipLaunchKernelGGL((k_cluster<false, 0>), dim3((unsigned)grid), dim3(kWG), 0, s, a);
    }
}

int cluster_capacity() { return kCap; }

// ------------------------------------------------------------- centroids
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

constexpr int kCWG = 256;      // threads per workgroup (k_seg_centroid)
constexpr int kHitCap = 1024;  // components per segment accumulated in LDS

// One workgroup per segment: exact integer moments of every component (LDS
// atomics, so the result does not depend on their order), then one hit per
// component at seg_off[k] + rank: X = sum(ToT x) / sum(ToT), same for Y and
// ToF; plain means when a component has no ToT at all.
__global__ __launch_bounds__(kCWG) void k_seg_centroid(ClusterArgs a) {
    // 64-bit weighted sums: a component of more than 2^32 / (1023 * 255)
    // = 16,464 pixels could overflow 32 bits
    __shared__ uint32_t CNT[kHitCap], TMIN[kHitCap], MINP[kHitCap];
    __shared__ unsigned long long W[kHitCap], SX[kHitCap], SY[kHitCap], ST[kHitCap];
    __shared__ uint32_t goff[kCWG + 1];
    const int tid = threadIdx.x;
    const uint32_t k = blockIdx.x;
    const uint64_t N = n_events(a);
    const uint64_t n_seg = (N + a.q - 1) / a.q;
    if (k == 0 && tid == 0) a.res->n_hits = a.seg_off[n_seg];
    if (k >= n_seg) return;
    Seg sg;
    if (!seg_bounds(a, k, N, sg)) return;
    const uint32_t cnt = a.seg_cnt[k], n = sg.n;
    if (cnt == 0) return;
    const uint64_t e0 = sg.e0, out0 = a.seg_off[k];
    const uint32_t ng = sg.g_hi - sg.g_lo;
    const bool goff_lds = ng <= (uint32_t)kCWG;
    if (goff_lds) {
        for (uint32_t i = tid; i <= ng; i += kCWG) goff[i] = a.grp_off[sg.g_lo + i];
    }
    if (cnt > n) {
        if (tid == 0) atomicOr(&a.res->err, (unsigned long long)kErrInternal);
        return;
    }
    if (cnt > (uint32_t)kHitCap) {
        // more components than LDS holds: 8 global words per component, in the
        // segment's own range of the scratch
        unsigned long long* acc = (unsigned long long*)a.g_acc + 8 * e0;
        for (uint32_t c = tid; c < cnt; c += kCWG) {
            unsigned long long* q = acc + 8 * c;
            q[0] = 0;
            q[1] = 0;
            q[2] = 0;
            q[3] = 0;
            q[4] = 0;
            q[5] = ~0ull;  // min t
            q[6] = ~0ull;  // min position
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kCWG) {
            const uint64_t pk = a.ev[e0 + i];
            const uint32_t rk = a.rank[e0 + i];
            if (rk >= cnt) {
                atomicOr(&a.res->err, (unsigned long long)kErrInternal);
                continue;
            }
            const uint32_t x = ev_x(pk), y = ev_y(pk), tot = ev_tot(pk), t = ev_t(pk);
            unsigned long long* q = acc + 8 * rk;
            atomicAdd(q + 0, (unsigned long long)tot);
            atomicAdd(q + 1, 1ull);
            atomicAdd(q + 2, (unsigned long long)(tot * x));
            atomicAdd(q + 3, (unsigned long long)(tot * y));
            atomicAdd(q + 4, (unsigned long long)time_term(a, tot, t));
            atomicMin(q + 5, (unsigned long long)t);
            atomicMin(q + 6, (unsigned long long)i);
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kCWG) {
            const uint32_t rk = a.rank[e0 + i];
            if (rk >= cnt) continue;
            unsigned long long* q = acc + 8 * rk;
            if (__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                const uint64_t pk = a.ev[e0 + i];
                atomicAdd(q + 2, (unsigned long long)ev_x(pk));
                atomicAdd(q + 3, (unsigned long long)ev_y(pk));
                atomicAdd(q + 4, (unsigned long long)time_term1(a, ev_tot(pk), ev_t(pk)));
            }
        }
        __syncthreads();
        for (uint32_t c = tid; c < cnt; c += kCWG) {
            unsigned long long* q = acc + 8 * c;
            unsigned long long v[7];
#pragma unroll
            for (int w = 0; w < 7; ++w)
                v[w] = __hip_atomic_load(q + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t p = (uint32_t)(e0 + v[6]);
            const uint32_t g = goff_lds ? sg.g_lo + group_of(goff, 0, ng, p)
                                        : group_of(a.grp_off, sg.g_lo, sg.g_hi, p);
            write_hit(a, out0 + c, g, v[0], v[1], v[2], v[3], v[4], (uint32_t)v[5],
                      gidx_of(a, e0 + v[6]));
        }
        return;
    }
    for (uint32_t c = tid; c < cnt; c += kCWG) {
        W[c] = 0;
        SX[c] = 0;
        SY[c] = 0;
        CNT[c] = 0;
        TMIN[c] = kNone32;
        MINP[c] = kNone32;
        ST[c] = 0;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kCWG) {
        const uint64_t pk = a.ev[e0 + i];
        const uint32_t rk = a.rank[e0 + i];
        if (rk >= cnt) {
            atomicOr(&a.res->err, (unsigned long long)kErrInternal);
            continue;
        }
        const uint32_t x = ev_x(pk), y = ev_y(pk), tot = ev_tot(pk), t = ev_t(pk);
        atomicAdd(&W[rk], (unsigned long long)tot);
        atomicAdd(&SX[rk], (unsigned long long)(tot * x));
        atomicAdd(&SY[rk], (unsigned long long)(tot * y));
        atomicAdd(&CNT[rk], 1u);
        atomicMin(&TMIN[rk], t);
        atomicMin(&MINP[rk], i);
        atomicAdd(&ST[rk], (unsigned long long)time_term(a, tot, t));
    }
    __syncthreads();
    // components without any ToT: plain means (the weighted sums are all
    // zero); the second pass runs only when such a component exists
    bool zero = false;
    for (uint32_t c = tid; c < cnt; c += kCWG) zero |= W[c] == 0;
    if (__syncthreads_or(zero)) {
        for (uint32_t i = tid; i < n; i += kCWG) {
            const uint32_t rk = a.rank[e0 + i];
            if (rk < cnt && W[rk] == 0) {
                const uint64_t pk = a.ev[e0 + i];
                atomicAdd(&SX[rk], (unsigned long long)ev_x(pk));
                atomicAdd(&SY[rk], (unsigned long long)ev_y(pk));
                atomicAdd(&ST[rk], (unsigned long long)time_term1(a, ev_tot(pk), ev_t(pk)));
            }
        }
        __syncthreads();
    }
    for (uint32_t c = tid; c < cnt; c += kCWG) {
        const uint32_t p = (uint32_t)(e0 + MINP[c]);
        const uint32_t g = goff_lds ? sg.g_lo + group_of(goff, 0, ng, p)
                                    : group_of(a.grp_off, sg.g_lo, sg.g_hi, p);
        write_hit(a, out0 + c, g, W[c], CNT[c], SX[c], SY[c], ST[c], TMIN[c],
                  gidx_of(a, e0 + MINP[c]));
    }
}

void launch_seg_centroid(const ClusterArgs& a, uint64_t grid, hipStream_t s) {
    if (grid == 0) return;
    hipLaunchKernelGGL(k_seg_centroid, dim3((unsigned)grid), dim3(kCWG), 0, s, a);
}

// ------------------------------------------------- paper local maxima
// The paper's own hits (Sec. V, Local Maxima and Centroiding): event i is a
// hit when no neighbour carries more ToT (Eqs. 6-7), ties going to the later
// event (its +0.001 i read as a tie-break by position), and its centroid is
// Eq. (9) over row i of A: itself and its direct neighbours.  Event mode, one
// workgroup per segment on the same image as k_cluster; the kernel runs
// twice: counting the maxima of every segment, then (after a prefix sum over
// segments) writing each maximum's hit at seg_off[k] + its rank.
// LDS byte layout of k_paper: image, then per event the packed word, the
// chain head and link, and the ToT
constexpr int kPOffEv = 32768;         // u64[kCap]
constexpr int kPOffChn = 49152;        // u32[kCap]
constexpr int kPOffNxt = 57344;        // u16[kCap]
constexpr int kPOffTot = 61440;        // u16[kCap]
constexpr int kLdsPaper = 65536;
static_assert(kPOffTot + 2 * kCap <= kLdsPaper, "paper layout");

// Local maxima of a segment of more than kCap events: per-event arrays in
// global scratch (pixel address, time, group start, ToT, slot-list link), the
// image of slot-list heads (u32) in LDS; the same decisions and moments as the
// LDS path.  Returns the segment's maximum count (count pass) after writing
// the hits (write pass).
template <bool kWrite>
__device__ uint32_t paper_big(const ClusterArgs& a, const uint64_t* __restrict__ trig,
                              uint8_t* lds, uint32_t* scan_tmp, const uint32_t* goff,
                              bool goff_lds, const Seg& sg, uint32_t k) {
    uint32_t* img = (uint32_t*)lds;  // u32[kH], all-ones = empty
    const uint64_t e0 = sg.e0;
    const uint32_t n = sg.n;
    uint32_t* xy = a.g_xy + e0;
    uint32_t* tt = a.g_t + e0;
    uint32_t* gs = a.g_sl + e0;
    uint32_t* tot = a.g_parent + e0;
    uint32_t* nxt = a.g_next + e0;
    const int tid = threadIdx.x;
    const int r = (int)a.dxy;
    const uint32_t dt = a.dt;
    unsigned long long* err = &a.res->err;
    {
        uint4* v = (uint4*)img;
        for (int i = tid; i < kH * 4 / 16; i += kWG) v[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
    }
    __syncthreads();
    const uint32_t ng = sg.g_hi - sg.g_lo;
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint32_t p = (uint32_t)(e0 + i);
        const uint32_t g = goff_lds ? sg.g_lo + group_of(goff, 0, ng, p)
                                    : group_of(a.grp_off, sg.g_lo, sg.g_hi, p);
        const Ev e = load_event<true>(a, e0 + i, g, e0, err);
        xy[i] = e.x | (e.y << 8);
        tt[i] = e.t;
        gs[i] = e.gs;
        tot[i] = a.soa.tot[orig_of(a, e0 + i)];
        nxt[i] = atomicExch(&img[slot_of(e.x, e.y)], i);
    }
    __syncthreads();
    // calls f(j) for every event j != i of the (2r+1)^2 box with an edge to i
    auto neighbours = [&](uint32_t i, auto&& f) {
        const uint32_t v = xy[i];
        const int x = (int)(v & 255u), y = (int)(v >> 8);
        const uint32_t t = tt[i], g = gs[i];
        bool ok = true;
        for (int dy = -r; dy <= r; ++dy) {
            const int ny = y + dy;
            if (ny < 0 || ny > 255) continue;
            for (int dx = -r; dx <= r; ++dx) {
                const int nx = x + dx;
                if (nx < 0 || nx > 255) continue;
                const uint32_t want = (uint32_t)nx | ((uint32_t)ny << 8);
                uint32_t j = img[slot_of((uint32_t)nx, (uint32_t)ny)], steps = 0;
                while (j != kNone32) {
                    if (j != i && xy[j] == want && gs[j] == g && absdiff(tt[j], t) <= dt) f(j);
                    if (++steps > n) {
                        ok = false;
                        break;
                    }
                    j = nxt[j];
                }
            }
        }
        if (!ok) atomicOr(err, (unsigned long long)kErrLoopChain);
    };
    uint32_t running = 0;
    const uint32_t rounds = (n + kWG - 1) / kWG;
    for (uint32_t rd = 0; rd < rounds; ++rd) {
        const uint32_t i = rd * kWG + tid;
        bool is_max = false;
        if (i < n) {
            is_max = true;
            const uint32_t ti = tot[i];
            neighbours(i, [&](uint32_t j) {
                const uint32_t tj = tot[j];
                if (tj > ti || (tj == ti && j > i)) is_max = false;
            });
        }
        uint32_t tot_r;
        const uint32_t rk = running + wg_flag_scan<kWG>(is_max, scan_tmp, &tot_r);
        if (kWrite && is_max) {
            // Eq. (9) over row i of A, exact integer moments
            const uint64_t oi = orig_of(a, e0 + i);
            const uint32_t sh = a.soa.shot[oi];
            const uint64_t T = trig[sh];
            uint64_t W = 0, cnt = 0, tmin = ~0ull;
            int64_t Sx = 0, Sy = 0, St = 0, Ux = 0, Uy = 0, Ut = 0;
            double Sw = 0.0, Uw = 0.0;
            auto add = [&](uint32_t j) {
                const uint64_t o = orig_of(a, e0 + j);
                const uint64_t toa = a.soa.toa[o];
                const uint32_t vj = xy[j];
                const int64_t x = (int64_t)(vj & 255u), y = (int64_t)(vj >> 8);
                const int64_t w = tot[j], tof = (int64_t)(toa - T);
                W += (uint64_t)w;
                Sx += w * x;
                Sy += w * y;
                St += w * tof;
                Ux += x;
                Uy += y;
                Ut += tof;
                if (a.walk) {
                    const double wk = (double)a.walk[w & 1023];
                    Sw += (double)w * wk;
                    Uw += wk;
                }
                ++cnt;
                tmin = toa < tmin ? toa : tmin;
            };
            add(i);
            neighbours(i, add);
            const uint64_t h = a.seg_off[k] + rk;
            if (h < a.hit_cap) {
                tpx_hit o;
                if (W) {
                    o.x = (float)((double)Sx / (double)W);
                    o.y = (float)((double)Sy / (double)W);
                    o.tof_ns = (float)((1.5625 * (double)St - Sw) / (double)W);
                } else {
                    o.x = (float)((double)Ux / (double)cnt);
                    o.y = (float)((double)Uy / (double)cnt);
                    o.tof_ns = (float)((1.5625 * (double)Ut - Uw) / (double)cnt);
                }
                o.npix = (uint32_t)cnt;
                o.shot = sh;
                o.label = oi;
                o.toa_first = tmin;
                o.tot_sum = (uint32_t)W;
                o.flags = W ? 0u : 1u;
                a.hits[h] = o;
            }
        }
        running += tot_r;
    }
    return running;
}

template <bool kWrite>
__global__ __launch_bounds__(kWG) void k_paper(ClusterArgs a, const uint64_t* __restrict__ trig) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsPaper];
    __shared__ uint32_t scan_tmp[kWG / 64 + 1];
    __shared__ uint32_t goff[kWG + 1];
    uint16_t* img = (uint16_t*)(lds + kOffImg);
    uint64_t* evs = (uint64_t*)(lds + kPOffEv);
    uint32_t* chn = (uint32_t*)(lds + kPOffChn);
    uint16_t* nxt = (uint16_t*)(lds + kPOffNxt);
    uint16_t* tt = (uint16_t*)(lds + kPOffTot);
    const int tid = threadIdx.x;
    const uint32_t k = blockIdx.x;
    const uint64_t N = n_events(a);
    const uint64_t n_seg = (N + a.q - 1) / a.q;
    if (k >= n_seg) return;
    Seg sg;
    if (!seg_bounds(a, k, N, sg)) return;
    const uint32_t n = sg.n;
    if (n == 0) {
        if (tid == 0 && !kWrite) a.seg_cnt[k] = 0;
        return;
    }
    if (n > (uint32_t)kCap) {
        // too large for LDS: the global-memory path
        const uint32_t ngb = sg.g_hi - sg.g_lo;
        const bool gl = ngb <= (uint32_t)kWG;
        if (gl)
            for (uint32_t i = tid; i <= ngb; i += kWG) goff[i] = a.grp_off[sg.g_lo + i];
        __syncthreads();
        const uint32_t cnt = paper_big<kWrite>(a, trig, lds, scan_tmp, goff, gl, sg, k);
        if (!kWrite && tid == 0) a.seg_cnt[k] = cnt;
        if (kWrite && k == 0 && tid == 0) a.res->n_hits = a.seg_off[n_seg];
        return;
    }
    const uint64_t e0 = sg.e0;
    const int r = (int)a.dxy;
    const uint32_t dt = a.dt;
    unsigned long long* err = &a.res->err;
    const uint32_t ng = sg.g_hi - sg.g_lo;
    const bool goff_lds = ng <= (uint32_t)kWG;
    if (goff_lds) {
        for (uint32_t i = tid; i <= ng; i += kWG) goff[i] = a.grp_off[sg.g_lo + i];
    }
    {
        uint4* v = (uint4*)img;
        for (int i = tid; i < kH * 2 / 16; i += kWG) v[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint32_t p = (uint32_t)(e0 + i);
        const uint32_t g = goff_lds ? sg.g_lo + group_of(goff, 0, ng, p)
                                    : group_of(a.grp_off, sg.g_lo, sg.g_hi, p);
        evs[i] = pack_lds(load_event<true>(a, e0 + i, g, e0, err));
        tt[i] = a.soa.tot[orig_of(a, e0 + i)];
        chn[i] = kNone32;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint64_t v = evs[i];
        img[slot_of((uint32_t)v & 255u, (uint32_t)(v >> 8) & 255u)] = (uint16_t)i;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kWG) {
        const uint64_t v = evs[i];
        const uint32_t w = img[slot_of((uint32_t)v & 255u, (uint32_t)(v >> 8) & 255u)];
        if (w != i) {
            const uint32_t old = atomicExch(&chn[w], i);
            nxt[i] = (uint16_t)(old == kNone32 ? kNone16 : old);
        }
    }
    __syncthreads();
    // maxima in position order, one workgroup-wide round at a time
    bool ok = true;
    uint32_t running = 0;
    const uint32_t rounds = (n + kWG - 1) / kWG;
    for (uint32_t rd = 0; rd < rounds; ++rd) {
        const uint32_t i = rd * kWG + tid;
        bool is_max = false;
        uint64_t v = 0;
        if (i < n) {
            v = evs[i];
            const uint32_t ti = tt[i];
            is_max = true;
            ok &= box_events<0>(img, chn, nxt, i, (int)(v & 255u), (int)((v >> 8) & 255u), r, n,
                                [&](uint32_t j, bool) {
                                    if (!is_edge(v, evs[j], r, dt)) return;
                                    const uint32_t tj = tt[j];
                                    if (tj > ti || (tj == ti && j > i)) is_max = false;
                                });
        }
        uint32_t tot_r;
        const uint32_t rk = running + wg_flag_scan<kWG>(is_max, scan_tmp, &tot_r);
        if (kWrite && is_max) {
            // Eq. (9) over row i of A, exact integer moments
            const uint64_t oi = orig_of(a, e0 + i);
            const uint32_t sh = a.soa.shot[oi];
            const uint64_t T = trig[sh];
            uint64_t W = 0, cnt = 0, tmin = ~0ull;
            int64_t Sx = 0, Sy = 0, St = 0, Ux = 0, Uy = 0, Ut = 0;
            double Sw = 0.0, Uw = 0.0;
            auto add = [&](uint32_t j) {
                const uint64_t o = orig_of(a, e0 + j);
                const uint64_t toa = a.soa.toa[o];
                const uint64_t vj = evs[j];
                const int64_t x = (int64_t)(vj & 255u), y = (int64_t)((vj >> 8) & 255u);
                const int64_t w = tt[j], tof = (int64_t)(toa - T);
                W += (uint64_t)w;
                Sx += w * x;
                Sy += w * y;
                St += w * tof;
                Ux += x;
                Uy += y;
                Ut += tof;
                if (a.walk) {
                    const double wk = (double)a.walk[w & 1023];
                    Sw += (double)w * wk;
                    Uw += wk;
                }
                ++cnt;
                tmin = toa < tmin ? toa : tmin;
            };
            add(i);
            ok &= box_events<0>(img, chn, nxt, i, (int)(v & 255u), (int)((v >> 8) & 255u), r, n,
                                [&](uint32_t j, bool) {
                                    if (is_edge(v, evs[j], r, dt)) add(j);
                                });
            const uint64_t h = a.seg_off[k] + rk;
            if (h < a.hit_cap) {
                tpx_hit o;
                if (W) {
                    o.x = (float)((double)Sx / (double)W);
                    o.y = (float)((double)Sy / (double)W);
                    o.tof_ns = (float)((1.5625 * (double)St - Sw) / (double)W);
                } else {
                    o.x = (float)((double)Ux / (double)cnt);
                    o.y = (float)((double)Uy / (double)cnt);
                    o.tof_ns = (float)((1.5625 * (double)Ut - Uw) / (double)cnt);
                }
                o.npix = (uint32_t)cnt;
                o.shot = sh;
                o.label = oi;
                o.toa_first = tmin;
                o.tot_sum = (uint32_t)W;
                o.flags = W ? 0u : 1u;
                a.hits[h] = o;
            }
        }
        running += tot_r;
    }
    if (!ok) atomicOr(err, (unsigned long long)kErrLoopChain);
    if (!kWrite && tid == 0) a.seg_cnt[k] = running;
    if (kWrite && k == 0 && tid == 0) a.res->n_hits = a.seg_off[n_seg];
}

void launch_paper(const ClusterArgs& a, const uint64_t* trig, bool write, uint64_t grid,
                  hipStream_t s) {
    if (grid == 0) return;
    if (write)
        hipLaunchKernelGGL(k_paper<true>, dim3((unsigned)grid), dim3(kWG), 0, s, a, trig);
    else
        hipLaunchKernelGGL(k_paper<false>, dim3((unsigned)grid), dim3(kWG), 0, s, a, trig);
}

}  // namespace tpx

namespace tpx {

// ================================================ fused stream-mode kernel
// Radius 1, stream mode: one workgroup per segment finds the segment's
// components (Eqs. 3-5 closed transitively), their exact integer moments and
// their hits (Eq. 9) without leaving the workgroup: the events are read from
// HBM once and the hits written once, into a staging buffer at the segment's
// own range (hit r of the segment at its first event index + r), from which
// a copy kernel moves them to their final place after a prefix sum of the
// segments' component counts.  No workgroup ever waits for another.
//
// LDS: an image of slot-list heads (u16, slot = (y mod 2^kYB, x)); every
// event is pushed on the list of its slot by a compare-and-swap of the 32-bit
// word that holds the slot, so a slot's list holds all its events after one
// pass.  Per event a 32-bit key, the
// union-find parent, the pixel address and ToT, and the list link (after the
// load no phase touches global memory until the hits are written).  The key holds the time of flight
// (16 bits; the kernel is used when every kept time of flight fits), the
// high bits of y that the slot does not hold, and the first position of the
// event's group (shot) in the segment: two events in slots of a 3x3 box are
// neighbours when their keys agree above the time bits (same group, exact
// row) and their times differ by at most the window.  After the unions the
// image region holds the per-component accumulators.
//
// Phases (each ends at a workgroup barrier reached by every thread):
//   1. load + push on the slot lists;
//   2. each event finds its neighbours in the backward half of its box (the
//      row above, the slot to its left, and earlier events of its own slot),
//      so every edge is seen once, keeps up to 8 of them in registers and
//      lowers the parents of both ends to the smaller end (LDS atomic
//      minimum): a min-neighbour forest;
//   3. pointer jumping, one pass that joins the two trees of every kept
//      edge by chains of atomic minima on tree roots, pointer jumping again
//      (the smallest position of each component, its label, is then every
//      member's parent);
//   4. ranks of the roots in position order;
//   5. moments per component (LDS atomics);
//   6. hits, staged.
// A segment over kSeg events keeps its per-event arrays in global scratch;
// a segment with more components than the accumulators hold sums them in
// global scratch; both in the same workgroup.

template <int kYB, int kNT, int kSeg>
struct FusedCfg {
    static constexpr int kSlots = 256 << kYB;      // u16 list heads
    static constexpr uint32_t kYMask = (1u << kYB) - 1u;
    static constexpr int kYHB = 8 - kYB;           // bits of y above the slot's
    // key: time (bits 0-15), a zero guard bit (16), then hi() from bit 17
    static constexpr int kHShift = 17;
    static constexpr int kGShift = kHShift + kYHB;  // group start above the time and y bits
    static constexpr int kE = kSeg / kNT;          // events per thread
    // edges kept in registers per event (more are found again by walking the
    // slot lists in every round): fewer where a thread holds many events
    static constexpr int kEdges = kE > 4 ? 4 : 8;
    static constexpr int kNW = kNT / 64;
    static constexpr int kOffKey = kSlots * 2;         // u32[kSeg]
    static constexpr int kOffPar = kOffKey + 4 * kSeg; // u32[kSeg]
    static constexpr int kOffXyt = kOffPar + 4 * kSeg; // u32[kSeg]: x | y << 8 | ToT << 16
    static constexpr int kOffNxt = kOffXyt + 4 * kSeg; // u16[kSeg]: list link, later root rank
    static constexpr int kBytes = kOffNxt + 2 * kSeg;
    // accumulators in the image region: u32 W, SX, SY, CNT, TMIN, P; u64 ST
    static constexpr int kHitCap = kSlots * 2 / 32;
    static_assert(kSeg % kNT == 0 && kSeg <= (1 << (32 - kGShift)) && kSeg < 65535,
                  "segment capacity");
    // the global-memory path keeps a u32 image of list heads in the same LDS
    static constexpr int kBigYB = (1024 << 6) <= kBytes ? 6 : (1024 << 5) <= kBytes ? 5 : 4;
    static constexpr int kBigSlots = 256 << kBigYB;
    static_assert(kBigSlots * 4 <= kBytes, "image of the global-memory path");
    __device__ static uint32_t big_slot(uint32_t x, uint32_t y) {
        return ((y & ((1u << kBigYB) - 1u)) << 8) | x;
    }
    __device__ static uint32_t slot(uint32_t x, uint32_t y) { return ((y & kYMask) << 8) | x; }
    // key bits above the time: group start and the high bits of y
    __device__ static uint32_t hi(uint32_t gs, uint32_t y) { return (gs << kYHB) | (y >> kYB); }
    // Offset that turns the neighbour test into one comparison: the key kj
    // has hi() = h and a time within dt of t exactly when
    // kj + off(h, t, dt) <= 2 dt (unsigned).  With equal hi() the sum is
    // tj - t + dt, in [0, 2 dt] exactly for the window and wrapped above it
    // when tj < t - dt; with unequal hi() it differs by a nonzero multiple
    // of 2^17 (mod 2^32) from a value in [-65535, 131070], which the guard
    // bit keeps out of [0, 2 dt] for any dt < 65536.
    __device__ static uint32_t off(uint32_t h, uint32_t t, uint32_t dt) {
        return dt - ((h << kHShift) | t);
    }
};

// Global accumulators of component c of the segment starting at e0: 8 words
// (W, count, Sx, Sy, St, min t, root position).
__device__ inline unsigned long long* gacc(const ClusterArgs& a, uint64_t e0, uint32_t c) {
    return (unsigned long long*)a.g_acc + 8 * (e0 + c);
}

__device__ inline void gacc_add(const ClusterArgs& a, unsigned long long* q, uint64_t pk) {
    const uint32_t x = ev_x(pk), y = ev_y(pk), tot = ev_tot(pk), t = ev_t(pk);
    atomicAdd(q + 0, (unsigned long long)tot);
    atomicAdd(q + 1, 1ull);
    atomicAdd(q + 2, (unsigned long long)(tot * x));
    atomicAdd(q + 3, (unsigned long long)(tot * y));
    atomicAdd(q + 4, (unsigned long long)time_term(a, tot, t));
    atomicMin(q + 5, (unsigned long long)t);
}

__device__ inline void gacc_add_plain(const ClusterArgs& a, unsigned long long* q, uint64_t pk) {
    atomicAdd(q + 2, (unsigned long long)ev_x(pk));
    atomicAdd(q + 3, (unsigned long long)ev_y(pk));
    atomicAdd(q + 4, (unsigned long long)time_term1(a, ev_tot(pk), ev_t(pk)));
}

__device__ inline unsigned long long gacc_ld(unsigned long long* q) {
    return __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Staged hit of component c (root = smallest position p in the segment).
__device__ inline void fused_emit(const ClusterArgs& a, const Seg& sg, const uint32_t* goff,
                                  bool goff_lds, uint32_t c, uint32_t p, uint64_t W, uint64_t cnt,
                                  uint64_t sx, uint64_t sy, uint64_t st, uint32_t tmin) {
    const uint32_t ng = sg.g_hi - sg.g_lo;
    const uint32_t pos = (uint32_t)(sg.e0 + p);
    const uint32_t g = goff_lds ? sg.g_lo + group_of(goff, 0, ng, pos)
                                : group_of(a.grp_off, sg.g_lo, sg.g_hi, pos);
    ClusterArgs b = a;  // the staging buffer stands in for the output
    b.hits = a.hits_tmp;
    b.hit_cap = ~0ull;
    write_hit(b, sg.e0 + c, g, W, cnt, sx, sy, st, tmin, gidx_of(a, sg.e0 + p));
}

// Components of a segment of more than C::kSeg events, per-event arrays in
// global scratch, the image in LDS.  Leaves the rank of every event's
// component in a.rank[e0 + i] and returns the component count.
template <class C, int kNT>
__device__ __forceinline__ uint32_t fused_big(const ClusterArgs& a, uint8_t* lds, uint32_t* scan_tmp,
                              const uint32_t* goff, bool goff_lds, const Seg& sg) {
    uint32_t* img = (uint32_t*)lds;
    const uint64_t e0 = sg.e0;
    const uint32_t n = sg.n, dt = a.dt;
    uint32_t* par = a.g_parent + e0;
    uint32_t* root = a.g_chain + e0;
    uint32_t* nxt = a.g_next + e0;
    uint32_t* tt = a.g_t + e0;
    uint32_t* gs = a.g_sl + e0;
    uint32_t* xy = a.g_xy + e0;
    const int tid = threadIdx.x;
    unsigned long long* err = &a.res->err;
    if (tid == 0) atomicAdd(&a.res->big_segments, 1ull);
    for (int i = tid; i < C::kBigSlots / 4; i += kNT)
        ((uint4*)img)[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kNT) {
        const uint32_t p = (uint32_t)(e0 + i);
        const uint32_t g = goff_lds ? sg.g_lo + group_of(goff, 0, sg.g_hi - sg.g_lo, p)
                                    : group_of(a.grp_off, sg.g_lo, sg.g_hi, p);
        const Ev e = load_event<false>(a, e0 + i, g, e0, err);
        par[i] = i;
        tt[i] = e.t;
        gs[i] = e.gs;
        xy[i] = e.x | (e.y << 8);
        nxt[i] = atomicExch(&img[C::big_slot(e.x, e.y)], i);
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kNT) {
        const uint32_t v = xy[i];
        const int x = (int)(v & 255u), y = (int)(v >> 8);
        const uint32_t t = tt[i], g = gs[i];
        for (int s = 0; s < 9; ++s) {
            const int nx = x + s % 3 - 1, ny = y + s / 3 - 1;
            if (nx < 0 || nx > 255 || ny < 0 || ny > 255) continue;
            uint32_t j = img[C::big_slot((uint32_t)nx, (uint32_t)ny)], steps = 0;
            while (j != kNone32) {
                if (j < i && gs[j] == g && absdiff(tt[j], t) <= dt &&
                    xy[j] == ((uint32_t)nx | ((uint32_t)ny << 8)))
                    uf_unite(par, i, j, n, err);
                if (++steps > n) {
                    atomicOr(err, (unsigned long long)kErrLoopChain);
                    break;
                }
                j = nxt[j];
            }
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kNT) root[i] = uf_find(par, i, n, err);
    __syncthreads();
    uint32_t running = 0;
    const uint32_t rounds = (n + kNT - 1) / kNT;
    for (uint32_t rd = 0; rd < rounds; ++rd) {
        const uint32_t i = rd * kNT + tid;
        uint32_t tot;
        const bool is_root = i < n && root[i] == i;
        const uint32_t rk = running + wg_flag_scan<kNT>(is_root, scan_tmp, &tot);
        if (is_root) par[i] = rk;  // parents are no longer needed: keep the rank
        running += tot;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kNT) a.rank[e0 + i] = par[root[i]];
    return running;
}

// kWaves: waves per SIMD the register allocation must allow (0: no bound)
// Segment k in one workgroup (every return below is taken by the whole
// workgroup).  With `defer`, a segment beyond the LDS capacity is not
// clustered here: its index is appended to a.defer_list for a later launch
// of a larger configuration.
template <int kYB, int kNT, int kSeg>
__device__ __forceinline__ void fused_segment(const ClusterArgs& a, uint32_t k, bool defer,
                                              uint8_t* lds, uint32_t* scan_tmp, uint32_t* goff) {
    using C = FusedCfg<kYB, kNT, kSeg>;
    constexpr int kE = C::kE;
    uint32_t* img = (uint32_t*)lds;  // as 32-bit words: two u16 heads each
    const uint16_t* head16 = (const uint16_t*)lds;
    uint32_t* key = (uint32_t*)(lds + C::kOffKey);
    uint32_t* par = (uint32_t*)(lds + C::kOffPar);
    uint32_t* xyt = (uint32_t*)(lds + C::kOffXyt);
    uint16_t* nxt = (uint16_t*)(lds + C::kOffNxt);
    // accumulators (after the unions)
    uint32_t* aW = img;
    uint32_t* aX = img + C::kHitCap;
    uint32_t* aY = img + 2 * C::kHitCap;
    uint32_t* aN = img + 3 * C::kHitCap;
    uint32_t* aT = img + 4 * C::kHitCap;
    uint32_t* aP = img + 5 * C::kHitCap;
    unsigned long long* aS = (unsigned long long*)(img + 6 * C::kHitCap);

    const int tid = threadIdx.x;
    unsigned long long* err = &a.res->err;
    const uint64_t N = n_events(a);
    const uint64_t n_seg = (N + a.q - 1) / a.q;
    if (k >= n_seg) return;
    Seg sg;
    if (!seg_bounds(a, k, N, sg)) {
        if (tid == 0) a.seg_cnt[k] = 0;
        return;
    }
    const uint32_t n = sg.n, dt = a.dt;
    const uint64_t e0 = sg.e0;
    if (n == 0) {
        if (tid == 0) a.seg_cnt[k] = 0;
        return;
    }
    if (defer && n > (uint32_t)kSeg) {
        if (tid == 0) a.defer_list[atomicAdd(&a.res->aux_ticket, 1ull)] = k;
        return;
    }
    const uint32_t ng = sg.g_hi - sg.g_lo;
    const bool goff_lds = ng <= (uint32_t)kNT;
    if (goff_lds)
        for (uint32_t i = tid; i <= ng; i += kNT) goff[i] = a.grp_off[sg.g_lo + i];

    uint32_t ncomp = 0;
    bool global_acc = false;  // moments in global scratch (ranks in a.rank)
    if (n > (uint32_t)kSeg) {
        __syncthreads();
        ncomp = fused_big<C, kNT>(a, lds, scan_tmp, goff, goff_lds, sg);
        global_acc = true;
    } else {
        // 1. load, push on the slot lists (with few events per thread, the
        // events are read while the image is cleared)
        constexpr bool kEarly = kE <= 4;
        uint64_t pkq[kEarly ? kE : 1];
        if constexpr (kEarly) {
#pragma unroll
            for (int q = 0; q < kE; ++q) {
                const uint32_t i = tid + q * kNT;
                pkq[q] = i < n ? a.ev[e0 + i] : 0ull;
            }
        }
        for (int i = tid; i < C::kSlots / 8; i += kNT)
            ((uint4*)img)[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t i = tid + q * kNT;
            if (i < n) {
                const uint64_t p = e0 + i;
                const uint32_t g = goff_lds ? sg.g_lo + group_of(goff, 0, ng, (uint32_t)p)
                                            : group_of(a.grp_off, sg.g_lo, sg.g_hi, (uint32_t)p);
                const uint32_t gs = (goff_lds ? goff[g - sg.g_lo] : a.grp_off[g]) - (uint32_t)e0;
                const uint64_t pk = kEarly ? pkq[kEarly ? q : 0] : a.ev[p];
                const uint32_t x = ev_x(pk), y = ev_y(pk);
                key[i] = (ev_t(pk) & 0xFFFFu) | (C::hi(gs, y) << C::kHShift);
                xyt[i] = x | (y << 8) | (ev_tot(pk) << 16);
                par[i] = i;
                // push i on its slot's list: swap it into the slot's half of
                // the 32-bit word (retried while the other half changes)
                const uint32_t sl = C::slot(x, y), sh = (sl & 1u) * 16u;
                uint32_t* w = img + (sl >> 1);
                uint32_t old = ald(w);
                for (uint32_t tries = 0;; ++tries) {
                    const uint32_t nw = (old & ~(0xFFFFu << sh)) | (i << sh);
                    uint32_t expect = old;
                    if (__hip_atomic_compare_exchange_strong(w, &expect, nw, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP) ||
                        tries > 2 * kSeg) {
                        if (tries > 2 * kSeg) atomicOr(err, (unsigned long long)kErrLoopUnite);
                        break;
                    }
                    old = expect;
                }
                nxt[i] = (uint16_t)((old >> sh) & 0xFFFFu);
            }
        }
        __syncthreads();
        // 2. neighbours in the backward half of the 3x3 box (the three slots
        // of the row above, the slot to the left and the event's own slot),
        // so that every edge is seen by exactly one of its ends (own slot:
        // by the later event).  The five list heads are read together, then
        // their keys and links, then those of the second events (two or
        // three LDS round trips when no list holds more than two events;
        // longer lists are walked afterwards).  Every event's parent becomes
        // the smallest of itself and its neighbours (atomic minimum from both
        // ends of each edge): a forest whose trees are mostly whole already.
        // The edges (up to C::kEdges per event) stay in registers.
        constexpr int kEd = C::kEdges, kNbW = kEd / 2;
        uint32_t nb[kE][kNbW];
        uint32_t meta[kE];  // edges found (at most 255 counted)
        bool ok = true;
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t i = tid + q * kNT;
            meta[q] = 0;
#pragma unroll
            for (int w = 0; w < kNbW; ++w) nb[q][w] = 0;
            if (i >= n) continue;
            const uint32_t xy = xyt[i];
            const int x = (int)(xy & 255u), y = (int)((xy >> 8) & 255u);
            const uint32_t ki = key[i];
            const uint32_t ti = ki & 0xFFFFu, gs = ki >> C::kGShift;
            const uint32_t off_up = C::off(C::hi(gs, (uint32_t)(y - 1)), ti, dt);
            const uint32_t off_row = C::off(C::hi(gs, (uint32_t)y), ti, dt);
            const uint32_t span = 2u * dt;
            constexpr int kDx[5] = {-1, 0, 1, -1, 0};
            constexpr int kDy[5] = {-1, -1, -1, 0, 0};
            uint32_t head[5];
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                const int nx = x + kDx[s], ny = y + kDy[s];
                const bool in = nx >= 0 && nx <= 255 && ny >= 0;
                head[s] = in ? head16[C::slot((uint32_t)nx, (uint32_t)ny)] : kNone16;
            }
            uint32_t hk[5], hn[5];
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                const uint32_t j = head[s] == kNone16 ? i : head[s];
                hk[s] = key[j];
                hn[s] = head[s] == kNone16 ? kNone16 : nxt[j];
            }
            uint32_t k2[5], n2[5];
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                const uint32_t j = hn[s] == kNone16 ? i : hn[s];
                k2[s] = key[j];
                n2[s] = hn[s] == kNone16 ? kNone16 : nxt[j];
            }
            uint32_t m = i, c = 0;
            // (events of other slots are never i itself; in its own slot
            // only earlier events count)
            auto take = [&](uint32_t j, uint32_t kj, int s) {
                if ((s < 4 || j < i) && kj + (s < 3 ? off_up : off_row) <= span) {
                    if (j < m) m = j;
                    if (s < 4) atomicMin(par + j, i);  // no-op when j < i (par[j] <= j)
                    // shift register of 16-bit links: the newest at the
                    // bottom, the oldest dropped past kEd
#pragma unroll
                    for (int w = kNbW - 1; w > 0; --w) nb[q][w] = (nb[q][w] << 16) | (nb[q][w - 1] >> 16);
                    nb[q][0] = (nb[q][0] << 16) | j;
                    ++c;
                }
            };
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                if (head[s] != kNone16) take(head[s], hk[s], s);
                if (hn[s] != kNone16) take(hn[s], k2[s], s);
            }
            bool longer = false;
#pragma unroll
            for (int s = 0; s < 5; ++s) longer |= n2[s] != kNone16;
            if (longer) {
                for (int s = 0; s < 5; ++s) {
                    uint32_t j = n2[s], steps = 0;
                    while (j != kNone16) {
                        take(j, key[j], s);
                        if (++steps > n) {
                            ok = false;
                            break;
                        }
                        j = nxt[j];
                    }
                }
            }
            meta[q] = c < 255 ? c : 255;
            if (m < i) atomicMin(par + i, m);
        }
        if (!ok) atomicOr(err, (unsigned long long)kErrLoopChain);
        __syncthreads();
        // 3. pointer jumping: every event then points at its tree's root
        // (a "jump root").  Then one pass over the edges: for an edge whose
        // ends read different parents h > l, an atomic minimum points h at l;
        // the old parent it returns is either h (h was a root: joined), l
        // (already joined) or a third node o, also a jump root, which is then
        // joined the same way with l (h -> l may have displaced h -> o, so o
        // and l must meet).  The larger node of each step is smaller than
        // the last, so every chain ends, and when all have ended every edge
        // joins one tree; only jump roots ever change their parent, and
        // parents only decrease, so the trees stay a forest whose roots are
        // the smallest positions of their components.  An event with more
        // edges than it keeps walks its lists instead.  A last pointer
        // jumping leaves every event pointing at its root.
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t i = tid + q * kNT;
            if (i >= n) continue;
            uint32_t p = ald(par + i), steps = 0;
            for (uint32_t nx; p != (nx = ald(par + p)) && ++steps <= n;) p = nx;
            ast(par + i, p);
        }
        __syncthreads();
        bool loop_err = false;
        auto join = [&](uint32_t u, uint32_t v) {
            uint32_t h = u < v ? v : u, l = u < v ? u : v;
            for (uint32_t st = 0;; ++st) {
                const uint32_t o = atomicMin(par + h, l);
                if (o == h || o == l) break;
                if (st > n) {
                    loop_err = true;
                    break;
                }
                h = o < l ? l : o;
                l = o < l ? o : l;
            }
        };
        uint32_t walks = 0;  // bit q: event tid + q kNT walks its lists
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t i = tid + q * kNT;
            if (i >= n) continue;
            const uint32_t cq = meta[q];
            if (cq > (uint32_t)kEd) {
                walks |= 1u << q;
                continue;
            }
            const uint32_t ri = ald(par + i);
            uint32_t rj[kEd];
#pragma unroll
            for (int t = 0; t < kEd; ++t) {
                const uint32_t j = (nb[q][t >> 1] >> ((t & 1) * 16)) & 0xFFFFu;
                rj[t] = (uint32_t)t < cq ? ald(par + j) : ri;
            }
#pragma unroll
            for (int t = 0; t < kEd; ++t)
                if (rj[t] != ri) join(ri, rj[t]);
        }
        // (one copy of the walk for all q: it reads everything from LDS)
#pragma unroll 1
        for (int q = 0; q < kE; ++q) {
            const uint32_t i = tid + q * kNT;
            if (!((walks >> q) & 1u)) continue;
            const uint32_t ri = ald(par + i);
            const uint32_t xy = xyt[i];
            const int x = (int)(xy & 255u), y = (int)((xy >> 8) & 255u);
            const uint32_t ki = key[i];
            const uint32_t ti = ki & 0xFFFFu, gs = ki >> C::kGShift;
            for (int s = 0; s < 5; ++s) {
                const int nx = x + (s == 3 ? -1 : s == 4 ? 0 : s - 1), ny = y - (s < 3 ? 1 : 0);
                if (nx < 0 || nx > 255 || ny < 0) continue;
                const uint32_t o = C::off(C::hi(gs, (uint32_t)ny), ti, dt);
                uint32_t j = head16[C::slot((uint32_t)nx, (uint32_t)ny)], steps = 0;
                while (j != kNone16) {
                    const uint32_t kj = key[j];
                    if ((s < 4 || j < i) && kj + o <= 2u * dt) {
                        const uint32_t r2 = ald(par + j);
                        if (r2 != ri) join(ri, r2);
                    }
                    if (++steps > n) break;
                    j = nxt[j];
                }
            }
        }
        if (loop_err) atomicOr(err, (unsigned long long)kErrLoopUnite);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t i = tid + q * kNT;
            if (i >= n) continue;
            uint32_t p = ald(par + i), steps = 0;
            for (uint32_t nx; p != (nx = ald(par + p)) && ++steps <= n;) p = nx;
            ast(par + i, p);
        }
        __syncthreads();
        // every parent is now its root; the image region becomes the accumulators
        for (int c = tid; c < C::kHitCap; c += kNT) {
            aW[c] = 0;
            aX[c] = 0;
            aY[c] = 0;
            aN[c] = 0;
            aT[c] = kNone32;
            aS[c] = 0;
        }
        __syncthreads();
        // 4. ranks of the roots in position order (thread t: positions kE t ..)
        {
            uint32_t cnt = 0;
#pragma unroll
            for (int q = 0; q < kE; ++q) {
                const uint32_t i = tid * kE + q;
                cnt += (i < n && par[i] == i) ? 1u : 0u;
            }
            uint32_t total;
            uint32_t r = wg_count_scan<kNT>(cnt, scan_tmp, &total);
#pragma unroll
            for (int q = 0; q < kE; ++q) {
                const uint32_t i = tid * kE + q;
                if (i < n && par[i] == i) {
                    nxt[i] = (uint16_t)r;  // the lists are no longer needed
                    if (r < (uint32_t)C::kHitCap) aP[r] = i;
                    ++r;
                }
            }
            ncomp = total;
        }
        __syncthreads();
        global_acc = ncomp > (uint32_t)C::kHitCap;
        if (global_acc) {
            // more components than the accumulators hold: ranks to a.rank
#pragma unroll
            for (int q = 0; q < kE; ++q) {
                const uint32_t i = tid + q * kNT;
                if (i < n) a.rank[e0 + i] = nxt[par[i]];
            }
        }
    }
    if (tid == 0) a.seg_cnt[k] = ncomp;

    if (global_acc) {
        // moments in the segment's own range of the global scratch
        for (uint32_t c = tid; c < ncomp; c += kNT) {
            unsigned long long* g = gacc(a, e0, c);
            g[0] = g[1] = g[2] = g[3] = g[4] = 0;
            g[5] = ~0ull;
            g[6] = ~0ull;
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kNT) {
            const uint32_t rk = a.rank[e0 + i];
            if (rk >= ncomp) {
                atomicOr(err, (unsigned long long)kErrInternal);
                continue;
            }
            unsigned long long* g = gacc(a, e0, rk);
            gacc_add(a, g, a.ev[e0 + i]);
            atomicMin(g + 6, (unsigned long long)i);
        }
        __syncthreads();
        bool zero = false;
        for (uint32_t c = tid; c < ncomp; c += kNT) zero |= gacc_ld(gacc(a, e0, c)) == 0;
        if (__syncthreads_or(zero)) {
            for (uint32_t i = tid; i < n; i += kNT) {
                const uint32_t rk = a.rank[e0 + i];
                if (rk < ncomp && gacc_ld(gacc(a, e0, rk)) == 0)
                    gacc_add_plain(a, gacc(a, e0, rk), a.ev[e0 + i]);
            }
            __syncthreads();
        }
        for (uint32_t c = tid; c < ncomp; c += kNT) {
            unsigned long long* g = gacc(a, e0, c);
            unsigned long long v[7];
#pragma unroll
            for (int w = 0; w < 7; ++w) v[w] = gacc_ld(g + w);
            fused_emit(a, sg, goff, goff_lds, c, (uint32_t)v[6], v[0], v[1], v[2], v[3], v[4],
                       (uint32_t)v[5]);
        }
        if (a.hit_index)
            for (uint32_t i = tid; i < n; i += kNT) a.hit_index[e0 + i] = a.rank[e0 + i];
        return;
    }

    // 5. moments (LDS atomics)
#pragma unroll
    for (int q = 0; q < kE; ++q) {
        const uint32_t i = tid + q * kNT;
        if (i >= n) continue;
        const uint32_t r = nxt[par[i]];
        const uint32_t v = xyt[i];
        const uint32_t x = v & 255u, y = (v >> 8) & 255u, tot = v >> 16, t = key[i] & 0xFFFFu;
        atomicAdd(&aW[r], tot);
        atomicAdd(&aX[r], tot * x);
        atomicAdd(&aY[r], tot * y);
        atomicAdd(&aN[r], 1u);
        atomicMin(&aT[r], t);
        atomicAdd(&aS[r], (unsigned long long)time_term(a, tot, t));
    }
    __syncthreads();
    bool zero = false;
    for (uint32_t c = tid; c < ncomp; c += kNT) zero |= aW[c] == 0;
    if (__syncthreads_or(zero)) {
        // components without any ToT: plain means (their weighted sums are 0)
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t i = tid + q * kNT;
            if (i >= n) continue;
            const uint32_t r = nxt[par[i]];
            if (aW[r] != 0) continue;
            const uint32_t v = xyt[i];
            atomicAdd(&aX[r], v & 255u);
            atomicAdd(&aY[r], (v >> 8) & 255u);
            atomicAdd(&aS[r], (unsigned long long)time_term1(a, v >> 16, key[i] & 0xFFFFu));
        }
        __syncthreads();
    }
    // 6. hits, staged at the segment's own range
    for (uint32_t c = tid; c < ncomp; c += kNT)
        fused_emit(a, sg, goff, goff_lds, c, aP[c], aW[c], aN[c], aX[c], aY[c], aS[c], aT[c]);
    if (a.hit_index) {
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t i = tid + q * kNT;
            if (i < n) a.hit_index[e0 + i] = nxt[par[i]];
        }
    }
}

// one workgroup per segment; with a.defer_list, segments beyond kSeg events
// are left to k_cluster_fused_list
template <int kYB, int kNT, int kSeg, int kWaves = 0>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(kWaves ? kWaves : 1)))
void k_cluster_fused(ClusterArgs a) {
    using C = FusedCfg<kYB, kNT, kSeg>;
    __shared__ __attribute__((aligned(16))) uint8_t lds[C::kBytes];
    __shared__ uint32_t scan_tmp[C::kNW + 1];
    __shared__ uint32_t goff[kNT + 1];
    fused_segment<kYB, kNT, kSeg>(a, blockIdx.x, a.defer_list != nullptr, lds, scan_tmp, goff);
}

// Persistent grid over the segments a previous k_cluster_fused launch
// deferred (a.res->aux_ticket of them in a.defer_list): each workgroup takes
// the next list entry from a ticket counter until the list is exhausted.  The
// ticket is broadcast through LDS between two barriers, so every thread of
// the workgroup leaves the loop in the same iteration; no workgroup waits for
// another.
template <int kYB, int kNT, int kSeg>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(kNT / 256)))
void k_cluster_fused_list(ClusterArgs a) {
    using C = FusedCfg<kYB, kNT, kSeg>;
    __shared__ __attribute__((aligned(16))) uint8_t lds[C::kBytes];
    __shared__ uint32_t scan_tmp[C::kNW + 1];
    __shared__ uint32_t goff[kNT + 1];
    __shared__ unsigned long long ticket;
    const unsigned long long n_list = a.res->aux_ticket;  // final: the deferring launch is done
    for (;;) {
        if (threadIdx.x == 0) ticket = atomicAdd(&a.res->seg_ticket, 1ull);
        __syncthreads();
        const unsigned long long t = ticket;
        if (t >= n_list) break;
        fused_segment<kYB, kNT, kSeg>(a, a.defer_list[t], false, lds, scan_tmp, goff);
        __syncthreads();  // LDS and the ticket are reused by the next segment
    }
}

// Staged hits to their final place: one wave per segment copies its hits
// (8-byte words: a hit record is 8-byte aligned) from the segment's staging
// range to seg_off[k]; with a hit index, the segment's events get their final
// hit.
constexpr int kCompactWG = 256;
// segment k by one wave (k = 0 also records the hit count)
__device__ __forceinline__ void hit_compact_wave(const ClusterArgs& a, uint64_t k) {
    const uint64_t N = n_events(a);
    const uint64_t n_seg = (N + a.q - 1) / a.q;
    const int lane = (int)__lane_id();
    if (k == 0 && lane == 0) a.res->n_hits = a.seg_off[n_seg];
    if (k >= n_seg) return;
    const uint32_t g_lo = a.seg_lo[k], g_hi = a.seg_lo[k + 1];
    const uint64_t e0 = a.grp_off[g_lo], e1 = a.grp_off[g_hi];
    if (g_hi < g_lo || e1 < e0 || e1 > N) return;  // reported by the cluster kernel
    const uint64_t cnt = a.seg_cnt[k], off = a.seg_off[k];
    const uint2* src = (const uint2*)(a.hits_tmp + e0);
    uint2* dst = (uint2*)(a.hits + off);
    static_assert(sizeof(tpx_hit) == 48, "hit record");
    uint64_t words = 6 * cnt;
    if (off >= a.hit_cap) words = 0;
    else if (off + cnt > a.hit_cap) words = 6 * (a.hit_cap - off);
    for (uint64_t w = lane; w < words; w += 64) dst[w] = src[w];
    if (a.hit_index)
        for (uint64_t i = e0 + lane; i < e1; i += 64) a.hit_index[i] += (uint32_t)off;
}
__global__ __launch_bounds__(kCompactWG) void k_hit_compact(ClusterArgs a) {
    hit_compact_wave(a, (uint64_t)blockIdx.x * (kCompactWG / 64) + (threadIdx.x >> 6));
}

struct FusedVariant {
    const char* name;
};
static const FusedVariant kFusedVariants[] = {
    {"image 256x32, 512 threads, 2048 events in LDS"},
    {"image 256x16, 512 threads, 2048 events in LDS, 8 waves per SIMD"},
    {"image 256x64, 512 threads, 2048 events in LDS"},
    {"image 256x32, 1024 threads, 2048 events in LDS"},
    {"image 256x64, 1024 threads, 8192 events in LDS"},
    {"routed: segments up to 2048 events as variant 1, larger ones by a persistent grid of "
     "variant 4's configuration"},
};

int fused_variants() { return (int)(sizeof(kFusedVariants) / sizeof(kFusedVariants[0])); }
const char* fused_variant_name(int v) {
    return v >= 0 && v < fused_variants() ? kFusedVariants[v].name : "?";
}

void launch_cluster_fused(const ClusterArgs& a0, uint64_t grid, int variant, uint32_t* defer_list,
                          uint32_t list_grid, hipStream_t s) {
    if (grid == 0) return;
    const dim3 g((unsigned)grid);
    ClusterArgs a = a0;
    a.defer_list = nullptr;
    if (variant == 5) {
        a.defer_list = defer_list;
        hipLaunchKernelGGL((k_cluster_fused<4, 512, 2048, 8>), g, dim3(512), 0, s, a);
        hipLaunchKernelGGL((k_cluster_fused_list<6, 1024, 8192>), dim3(list_grid ? list_grid : 1),
                           dim3(1024), 0, s, a);
        return;
    }
    switch (variant) {
    case 1: hipLaunchKernelGGL((k_cluster_fused<4, 512, 2048, 8>), g, dim3(512), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_cluster_fused<6, 512, 2048>), g, dim3(512), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_cluster_fused<5, 1024, 2048>), g, dim3(1024), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_cluster_fused<6, 1024, 8192>), g, dim3(1024), 0, s, a); break;
    default: hipLaunchKernelGGL((k_cluster_fused<5, 512, 2048>), g, dim3(512), 0, s, a); break;
    }
}

void launch_hit_compact(const ClusterArgs& a, uint64_t grid, hipStream_t s) {
    if (grid == 0) return;
    const uint64_t blocks = (grid + kCompactWG / 64 - 1) / (kCompactWG / 64);
    hipLaunchKernelGGL(k_hit_compact, dim3((unsigned)blocks), dim3(kCompactWG), 0, s, a);
}

}  // namespace tpx

namespace tpx {

// ============================================== persistent chunk kernel
// One launch for the whole fast stream path of a chunk (decode, unwrap,
// shot assignment and compaction, grouping, components, moments, hits,
// carry): a persistent grid whose workgroups take work items from a ticket
// counter.  Items are numbered in dependency order, and an item waits only
// for the done-counters of items with smaller tickets, which are held by
// workgroups that are already running; so the grid needs no co-residency and
// every wait ends (each one is also bounded).  Every item waits for each
// item it reads from directly (not only through a chain that an empty range
// of items would break, as with a chunk of no tiles).  Items:
//   [0, T)        tile summaries                       -> kDoneSum
//   T             prefix over the tiles (one workgroup: entry states,
//                 trigger unwrap, results zeroed, shot counts cleared,
//                 carried events in)                    -> kDonePre
//   [T+1, 2T+1)   shot assignment of each tile, staged  -> kDoneAsg
//   2T+1          prefix of the tiles' kept counts      -> kDoneTsc
//   [2T+2, 3T+2)  placement of each tile's kept events  -> kDonePlc
//   3T+2          statistics, shot offsets, close rule, segment table
//                                                       -> kDoneGrp
//   [3T+3, +S)    one segment each (fused components, moments, hits)
//                                                       -> kDoneCl
//   3T+3+S        prefix of the segments' hit counts, carry of open shots
//                                                       -> kDoneFin
//   then          hit compaction, eight segments per item.
// The last workgroup to leave resets the counters for the next launch.
constexpr int kChunkThreads = 512;
enum : int { kQTicket = 0, kQExit, kDoneSum, kDonePre, kDoneAsg, kDoneTsc, kDonePlc, kDoneGrp,
             kDoneCl, kDoneFin, kQWords };
using ChunkCfg = FusedCfg<4, kChunkThreads, 2048>;

union ChunkLds {
    AssignLds<kChunkThreads> as;
    struct {
        __attribute__((aligned(16))) uint8_t lds[ChunkCfg::kBytes];
        uint32_t scan_tmp[ChunkCfg::kNW + 1];
        uint32_t goff[kChunkThreads + 1];
    } cl;
    struct {
        RunSum wbuf[kChunkThreads / 64];
        TileAcc abuf[kChunkThreads / 64];
        uint32_t tmp[kChunkThreads / 64 + 1];
        unsigned long long st[kChunkThreads / 64][8];
        uint64_t bc[2];
    } w;
};

// exclusive in-order fold of one TileAcc per thread of the workgroup
__device__ inline TileAcc chunk_acc_exscan(TileAcc v, TileAcc* wbuf, uint64_t jump, TileAcc* all) {
    constexpr int NW = kChunkThreads / 64;
    const TileAcc inc = wave_acc_inscan(v, jump);
    const TileAcc ex = wave_acc_shift1(inc);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 63) wbuf[w] = inc;
    __syncthreads();
    TileAcc pre = acc_empty(), tot = acc_empty();
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const TileAcc c = wbuf[k];
        if (k < w) pre = acc_combine(pre, c, jump);
        tot = acc_combine(tot, c, jump);
    }
    __syncthreads();
    *all = tot;
    return acc_combine(pre, ex, jump);
}

// out[0..n] = exclusive prefix of in[0..n), out[n] = total, by one workgroup
__device__ inline void chunk_scan_u32(const uint32_t* in, uint32_t* out, uint64_t n,
                                      uint32_t* tmp) {
    uint32_t run = 0;
    for (uint64_t base = 0; base < n; base += kChunkThreads) {
        const uint64_t i = base + threadIdx.x;
        const uint32_t v = i < n ? in[i] : 0u;
        uint32_t tot;
        const uint32_t p = wg_count_scan<kChunkThreads>(v, tmp, &tot);
        if (i < n) out[i] = run + p;
        run += tot;
    }
    if (threadIdx.x == 0) out[n] = run;
}

// thread 0 waits until counter q reaches `target`; false after the bound.
// Relaxed polls with a growing pause (many workgroups may wait on one
// counter), then one acquire.
__device__ inline bool chunk_wait(unsigned int* q, unsigned int target) {
    __shared__ int ok;
    if (threadIdx.x == 0) {
        int good = 1;
        for (uint32_t spin = 0;
             __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++spin) {
            if (spin >= (1u << 22)) {
                good = 0;
                break;
            }
            if (spin < 16) __builtin_amdgcn_s_sleep(1);
            else if (spin < 256) __builtin_amdgcn_s_sleep(4);
            else __builtin_amdgcn_s_sleep(16);
        }
        (void)__hip_atomic_load(q, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        ok = good;
    }
    __syncthreads();
    const bool r = ok != 0;
    __syncthreads();  // every thread has read `ok` before the next wait writes it
    __threadfence();
    return r;
}

__device__ inline void chunk_signal(unsigned int* q) {
    __syncthreads();  // every thread's writes of the item are done
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_fetch_add(q, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The arguments come through a pointer to device memory: passed by value,
// this large a block would be copied to scratch memory in this kernel.  Two
// waves per SIMD (one workgroup per CU): the items' code then needs no
// spills, which measured faster for the small chunks this launch serves
// than four waves with spills.
__global__ __launch_bounds__(kChunkThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_stream_chunk(const ChunkArgs* __restrict__ pp) {
    const ChunkArgs& p = *pp;
    __shared__ ChunkLds L;
    __shared__ uint32_t s_ticket;
    const uint32_t tid = threadIdx.x;
    unsigned int* q = p.qs;
    DevResults* res = p.a.res;
    const uint32_t T = p.ntiles, S = p.seg_grid, C = (S + 7) / 8;
    const uint32_t total = 3 * T + 4 + S + C;
    for (;;) {
        if (tid == 0) s_ticket = __hip_atomic_fetch_add(q + kQTicket, 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t t = s_ticket;
        __syncthreads();
        if (t >= total) break;
        if (t < T) {
            tile_summary_body(p.a.pk, p.a.n, p.a.sub, p.a.jump, p.sums, p.tdc_slot, t, L.w.wbuf,
                              L.w.tmp);
            chunk_signal(q + kDoneSum);
        } else if (t == T) {
            const bool ok = chunk_wait(q + kDoneSum, T);
            // results of the call start at zero (no earlier item writes them)
            for (uint32_t i = tid; i < sizeof(DevResults) / 8; i += kChunkThreads)
                ((unsigned long long*)res)[i] = 0;
            __syncthreads();
            if (!ok && tid == 0) atomicOr(&res->err, (unsigned long long)kErrSpin);
            TileAcc v = tid < T ? p.sums[tid] : acc_empty();
            if (tid == 0) v = acc_combine(p.init, v, p.a.jump);
            TileAcc all;
            TileAcc ex = chunk_acc_exscan(v, L.w.abuf, p.a.jump, &all);
            if (tid == 0) ex = p.init;
            if (tid == 0) {
                res->pix_epoch_end = p.pe0 + all.pix.sum;
                res->tdc_epoch_end = p.te0 + all.tdc.sum;
                res->pix_last_end = all.pix.last;
                res->tdc_last_end = all.tdc.last;
                res->pix_has_end = all.pix.count > 0;
                res->tdc_has_end = all.tdc.count > 0;
                res->n_trig = all.ntrig - p.init.ntrig;
            }
            if (tid < T)
                unwrap_tile(ex, p.init.ntrig, tid, p.sums, p.tdc_slot, p.pe0, p.te0, p.a.jump,
                            p.entries, p.tab_new, res);
            // shot counts of the window and this call's triggers start at zero,
            // then the carried events count in
            const uint64_t rows = p.a.n_win + (all.ntrig - p.init.ntrig) + 2;
            for (uint64_t i = tid; i < rows; i += kChunkThreads) p.a.shot_cnt[i] = 0;
            __syncthreads();
            carry_in_range(p.c_ev_in, p.c_shot_in, p.n_carry, p.carry_rebase, p.ev, nullptr,
                           p.a.shot_cnt, tid, kChunkThreads);
            chunk_signal(q + kDonePre);
        } else if (t < 2 * T + 1) {
            if (!chunk_wait(q + kDonePre, 1) && tid == 0)
                atomicOr(&res->err, (unsigned long long)kErrSpin);
            assign_body<false, true, kChunkThreads>(p.a, t - (T + 1), L.as);
            chunk_signal(q + kDoneAsg);
        } else if (t == 2 * T + 1) {
            // (the prefix too: with no tiles there is no assignment to wait for)
            if (!(chunk_wait(q + kDonePre, 1) & chunk_wait(q + kDoneAsg, T)) && tid == 0)
                atomicOr(&res->err, (unsigned long long)kErrSpin);
            chunk_scan_u32(p.a.tile_cnt, p.tile_off, T, L.w.tmp);
            chunk_signal(q + kDoneTsc);
        } else if (t < 3 * T + 2) {
            if (!chunk_wait(q + kDoneTsc, 1) && tid == 0)
                atomicOr(&res->err, (unsigned long long)kErrSpin);
            place_tile(p.a, p.tile_off, p.ev, p.n_carry, p.ev_cap, nullptr, T, t - (2 * T + 2),
                       kChunkThreads);
            chunk_signal(q + kDonePlc);
        } else if (t == 3 * T + 2) {
            if (!(chunk_wait(q + kDoneTsc, 1) & chunk_wait(q + kDonePlc, T)) && tid == 0)
                atomicOr(&res->err, (unsigned long long)kErrSpin);
            // statistics of the tiles
            unsigned long long v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (tid < T) {
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] = p.a.tile_stat[8ull * tid + k];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                for (int d = 32; d > 0; d >>= 1) {
                    const unsigned long long o = __shfl_xor(v[k], d, 64);
                    v[k] = k < 7 ? v[k] + o : max(v[k], o);
                }
            if (__lane_id() == 0)
                for (int k = 0; k < 8; ++k) L.w.st[tid >> 6][k] = v[k];
            __syncthreads();
            if (tid == 0) {
                unsigned long long x[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                for (int w = 0; w < kChunkThreads / 64; ++w)
                    for (int k = 0; k < 8; ++k)
                        x[k] = k < 7 ? x[k] + L.w.st[w][k] : max(x[k], L.w.st[w][k]);
                res->n_pixels += x[0];
                res->n_other += x[1];
                res->n_pre_trigger += x[2];
                res->n_tof_cut += x[3];
                res->n_late_drop += x[4];
                res->n_pix_wraps += x[5];
                res->n_pix_backjumps += x[6];
                res->max_t_plus1 = max(res->max_t_plus1, x[7]);
                res->n_groups = p.a.n_win + res->n_trig;
                L.w.bc[0] = res->n_groups;
            }
            __syncthreads();
            const uint64_t G = L.w.bc[0];
            uint32_t* shot_off = const_cast<uint32_t*>(p.c.grp_off);
            chunk_scan_u32(p.a.shot_cnt, shot_off, G, L.w.tmp);
            __syncthreads();
            if (tid == 0)
                close_rule(p.a.tab, &res->n_trig, p.a.n_win, p.a.first_open, p.flush,
                           p.max_t_plus1_prev, p.a.tof_max, p.slack, p.c.grp_off, res);
            __syncthreads();
            seg_table_range(p.c.grp_off, p.c.n_grp_dev, p.c.n_ev_dev, p.c.skip, p.c.q,
                            const_cast<uint32_t*>(p.c.seg_lo), res, tid, kChunkThreads);
            chunk_signal(q + kDoneGrp);
        } else if (t < 3 * T + 3 + S) {
            if (!chunk_wait(q + kDoneGrp, 1) && tid == 0)
                atomicOr(&res->err, (unsigned long long)kErrSpin);
            fused_segment<4, kChunkThreads, 2048>(p.c, t - (3 * T + 3), false, L.cl.lds,
                                                  L.cl.scan_tmp, L.cl.goff);
            chunk_signal(q + kDoneCl);
        } else if (t == 3 * T + 3 + S) {
            if (!(chunk_wait(q + kDoneGrp, 1) & chunk_wait(q + kDoneCl, S)) && tid == 0)
                atomicOr(&res->err, (unsigned long long)kErrSpin);
            chunk_scan_u32(p.c.seg_cnt, const_cast<uint32_t*>(p.c.seg_off), res->n_seg, L.w.tmp);
            carry_out_range(p.ev, nullptr, nullptr, p.c.grp_off, &res->n_groups, &res->n_close_ev,
                            &res->n_kept, p.c_gidx_in, p.n_carry, p.c.ev_base, p.c_ev_out,
                            p.c_shot_out, p.c_gidx_out, p.carry_cap, res, tid, kChunkThreads);
            chunk_signal(q + kDoneFin);
        } else {
            if (!chunk_wait(q + kDoneFin, 1) && tid == 0)
                atomicOr(&res->err, (unsigned long long)kErrSpin);
            hit_compact_wave(p.c, (uint64_t)(t - (3 * T + 4 + S)) * 8 + (tid >> 6));
        }
        __syncthreads();  // LDS and the ticket are reused by the next item
    }
    if (tid == 0) {
        const unsigned int e = __hip_atomic_fetch_add(q + kQExit, 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        if (e == gridDim.x - 1)  // every other workgroup has left: reset for the next launch
            for (int i = 0; i < kQWords; ++i)
                __hip_atomic_store(q + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

uint32_t chunk_max_tiles() { return kChunkThreads; }
uint32_t chunk_queue_words() { return kQWords; }

void launch_stream_chunk(const ChunkArgs& p, const ChunkArgs* p_dev, uint32_t grid, hipStream_t s) {
    const uint64_t total = 3ull * p.ntiles + 4 + p.seg_grid + (p.seg_grid + 7) / 8;
    const uint64_t want = grid ? grid : 1;
    const uint32_t g = (uint32_t)(total < want ? total : want);
    hipLaunchKernelGGL(k_stream_chunk, dim3(g), dim3(kChunkThreads), 0, s, p_dev);
}

}  // namespace tpx
