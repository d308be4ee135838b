/*
 * tpx_oracle.c -- reference implementation of the TimePix3 VMI hot path,
 * written to be read and checked, not to be fast.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load, call or run this file.  The library
 * never does; it shares no code, header, table or constant with it.
 *
 * What it computes (arXiv 2603.04942, "Fast array-based particle coincidence
 * detection in a TimePix3-based velocity map imaging instrument"):
 *
 *   1. decode   each 64-bit word into a pixel (x, y, ToT, 34-bit arrival
 *               tick), a laser trigger (36-bit tick) or "other" (Sec. III;
 *               the bit layout is not in the paper, see decode_word below);
 *   2. unwrap   pixel and trigger times separately: a drop of more than the
 *               jump threshold against the previous word of the same stream
 *               adds one wrap period, a rise of more than it removes one
 *               (Sec. IV, ToA Unwrapping, including the late-reporter case);
 *   3. assign   each pixel to the latest trigger at or before it and drop it
 *               when its time of flight exceeds the cut (Sec. IV, Eliminating
 *               Background Counts);
 *   4. cluster  the kept pixels: i and j are neighbours when they belong to
 *               the same shot and |dx| <= r, |dy| <= r, |dt| <= r_t, which is
 *               the Hadamard product of the three per-axis threshold matrices
 *               (Sec. V, Neighborhoods, Eqs. 3-5); a hit is a connected
 *               component of that graph (the transitive closure of A) and is
 *               labelled by its smallest event index;
 *   5. centroid each hit with ToT as the mass, Eq. (8)-(9) evaluated on the
 *               closure: X = sum(ToT x) / sum(ToT), same for Y and ToF
 *               (Sec. V, Centroiding).  An optional time-walk table
 *               Delta ToF(ToT) (Eq. 1) is subtracted from each pixel's ToF.
 *
 * Integer moments are exact (int64); the three divisions are done in double.
 *
 * The paper's own hit definition is here too (orc_local_maxima): a pixel is
 * a hit when its ToT exceeds that of every neighbour (Sec. V, Local Maxima,
 * Eqs. 6-7), and its centroid is Eq. (9) over its own row of A, i.e. its
 * direct neighbours, not the closure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ECAPACITY (-2)
#define ORC_ESTREAM (-3)
#define ORC_ENOMEM (-5)

/* one tick = 1.5625 ns = 256 units of the chip's 25/4096 ns (Sec. IV) */
static const double ORC_TICK_NS = 1.5625;
/* 2^42 and 2^44 chip units (Sec. IV) expressed in 1.5625 ns ticks */
static const uint64_t ORC_PIX_PERIOD = 1ull << 34;
static const uint64_t ORC_TDC_PERIOD = 1ull << 36;

enum { ORC_PIXEL = 0, ORC_TRIGGER = 1, ORC_OTHER = 2 };

typedef struct {
    uint32_t dxy;           /* spatial radius, Chebyshev; 1 = 8-neighbours      */
    uint32_t dt_ticks;      /* |ToA difference| allowed inside a hit, inclusive */
    uint32_t tof_max_ticks; /* keep a pixel when its ToF <= this                */
    uint32_t trig_subtype;  /* TDC subtype nibble that marks a laser trigger    */
    uint64_t jump_ticks;    /* unwrap threshold                                  */
    int64_t pix_epoch0;     /* wrap count in force before the first pixel        */
    int64_t tdc_epoch0;     /* wrap count in force before the first trigger      */
    const double* walk_ns;  /* NULL, or 1024 values of Delta ToF(ToT) in ns      */
} orc_params;

typedef struct {
    uint64_t n_packets, n_pixels, n_tdc, n_other, n_pre_trigger, n_tof_cut,
        n_events, n_hits, n_pix_wraps, n_pix_backjumps, n_tdc_wraps,
        n_tdc_backjumps;
} orc_stats;

typedef struct {
    double x, y, tof_ns;
    uint64_t shot, label, toa_first, npix, tot_sum;
    uint32_t flags, pad;
} orc_hit;

/* ---------------------------------------------------------------- decode */

/* Bit layout (the paper does not print one; this is the project's reading
 * of the TPX3 stream):
 *   pixel  0xB | x>>1 (7) | y>>2 (6) | pix (3) | coarse ToA (14) | ToT (10)
 *              | fine ToA (4) | spidr (16);  x = 2*(x>>1) + (pix>>2),
 *              y = 4*(y>>2) + (pix&3), tick = ((spidr<<14 | ToA) << 4) - fine
 *              modulo 2^34
 *   TDC    0x6 | subtype (4) | counter (12) | timestamp (35, 3.125 ns) | ...;
 *              tick = 2 * timestamp modulo 2^36
 */
int orc_decode_word(uint64_t w, uint32_t trig_subtype, uint32_t* kind,
                    uint32_t* x, uint32_t* y, uint32_t* tot, uint64_t* raw)
{
    uint32_t header = (uint32_t)(w >> 60);
    *x = *y = *tot = 0;
    *raw = 0;
    if (header == 0xB) {
        uint32_t dcol = (uint32_t)((w >> 53) & 0x7F);
        uint32_t spix = (uint32_t)((w >> 47) & 0x3F);
        uint32_t pix = (uint32_t)((w >> 44) & 0x7);
        uint64_t toa = (w >> 30) & 0x3FFF;
        uint64_t ftoa = (w >> 16) & 0xF;
        uint64_t spidr = w & 0xFFFF;
        uint64_t coarse = (spidr << 14) | toa;
        *x = 2 * dcol + (pix >> 2);
        *y = 4 * spix + (pix & 3);
        *tot = (uint32_t)((w >> 20) & 0x3FF);
        *raw = ((coarse << 4) - ftoa) & (ORC_PIX_PERIOD - 1);
        *kind = ORC_PIXEL;
        return 0;
    }
    if (header == 0x6 && (uint32_t)((w >> 56) & 0xF) == trig_subtype) {
        uint64_t stamp = (w >> 9) & ((1ull << 35) - 1);
        *raw = (2 * stamp) & (ORC_TDC_PERIOD - 1);
        *kind = ORC_TRIGGER;
        return 0;
    }
    *kind = ORC_OTHER;
    return 0;
}

/* ---------------------------------------------------------------- unwrap */

typedef struct {
    int have_prev;
    uint64_t prev_raw;
    int64_t epoch;
    uint64_t period;
    uint64_t jump;
    uint64_t* n_wraps;
    uint64_t* n_back;
} orc_unwrapper;

/* Sec. IV: a drop of more than the threshold against the previous value of
 * the same stream means the counter wrapped (one period more from here on);
 * a rise of more than the threshold is a late reporter from before the wrap
 * (one period less).  Returns the unwrapped tick, or -1 when the wrap count
 * would go negative. */
static int64_t orc_unwrap(orc_unwrapper* u, uint64_t raw)
{
    if (u->have_prev) {
        int64_t d = (int64_t)raw - (int64_t)u->prev_raw;
        if (d < -(int64_t)u->jump) {
            u->epoch += 1;
            (*u->n_wraps)++;
        } else if (d > (int64_t)u->jump) {
            u->epoch -= 1;
            (*u->n_back)++;
        }
    }
    u->have_prev = 1;
    u->prev_raw = raw;
    if (u->epoch < 0) return -1;
    return (int64_t)(raw + (uint64_t)u->epoch * u->period);
}

/* Steps 1-3.  Events come out in stream order.  t_out (may be NULL) receives
 * the unwrapped tick of every pixel and trigger word (0 for others). */
int orc_decode(const uint64_t* pk, size_t n, const orc_params* p,
               uint16_t* ex, uint16_t* ey, uint16_t* etot, uint32_t* eshot,
               uint64_t* etoa, size_t ev_cap, size_t* n_ev,
               uint64_t* trig, size_t trig_cap, size_t* n_trig,
               int64_t* t_out, orc_stats* st)
{
    memset(st, 0, sizeof(*st));
    st->n_packets = n;
    *n_ev = 0;
    *n_trig = 0;
    if (p->pix_epoch0 < 0 || p->tdc_epoch0 < 0) return ORC_EINVAL;

    int64_t* t = (int64_t*)malloc((n ? n : 1) * sizeof(int64_t));
    uint8_t* kind = (uint8_t*)malloc(n ? n : 1);
    if (!t || !kind) { free(t); free(kind); return ORC_ENOMEM; }

    orc_unwrapper up = {0, 0, p->pix_epoch0, ORC_PIX_PERIOD, p->jump_ticks,
                        &st->n_pix_wraps, &st->n_pix_backjumps};
    orc_unwrapper ut = {0, 0, p->tdc_epoch0, ORC_TDC_PERIOD, p->jump_ticks,
                        &st->n_tdc_wraps, &st->n_tdc_backjumps};
    size_t nt = 0;
    uint64_t last_trig = 0;
    int rc = ORC_OK;
    for (size_t i = 0; i < n; ++i) {
        uint32_t k, x, y, tot;
        uint64_t raw;
        orc_decode_word(pk[i], p->trig_subtype, &k, &x, &y, &tot, &raw);
        kind[i] = (uint8_t)k;
        t[i] = 0;
        if (k == ORC_PIXEL) {
            st->n_pixels++;
            t[i] = orc_unwrap(&up, raw);
            if (t[i] < 0) { rc = ORC_ESTREAM; break; }
        } else if (k == ORC_TRIGGER) {
            st->n_tdc++;
            t[i] = orc_unwrap(&ut, raw);
            if (t[i] < 0) { rc = ORC_ESTREAM; break; }
            if (nt > 0 && (uint64_t)t[i] < last_trig) { rc = ORC_ESTREAM; break; }
            last_trig = (uint64_t)t[i];
            if (nt < trig_cap) trig[nt] = last_trig;
            else rc = ORC_ECAPACITY;
            nt++;
        } else {
            st->n_other++;
        }
    }
    *n_trig = nt;
    if (t_out && rc == ORC_OK) memcpy(t_out, t, n * sizeof(int64_t));
    if (rc != ORC_OK) { free(t); free(kind); return rc; }

    /* step 3: the most recent trigger by time, T[s] <= t < T[s+1] */
    size_t ne = 0;
    for (size_t i = 0; i < n; ++i) {
        if (kind[i] != ORC_PIXEL) continue;
        uint64_t ti = (uint64_t)t[i];
        size_t lo = 0, hi = nt; /* upper_bound: first T > t */
        while (lo < hi) {
            size_t mid = lo + (hi - lo) / 2;
            if (trig[mid] <= ti) lo = mid + 1; else hi = mid;
        }
        if (lo == 0) { st->n_pre_trigger++; continue; }
        size_t s = lo - 1;
        uint64_t tof = ti - trig[s];
        if (tof > p->tof_max_ticks) { st->n_tof_cut++; continue; }
        if (ne < ev_cap) {
            uint32_t k, x, y, tot;
            uint64_t raw;
            orc_decode_word(pk[i], p->trig_subtype, &k, &x, &y, &tot, &raw);
            ex[ne] = (uint16_t)x;
            ey[ne] = (uint16_t)y;
            etot[ne] = (uint16_t)tot;
            eshot[ne] = (uint32_t)s;
            etoa[ne] = ti;
        }
        ne++;
    }
    st->n_events = ne;
    *n_ev = ne;
    free(t);
    free(kind);
    return ne > ev_cap ? ORC_ECAPACITY : ORC_OK;
}

/* --------------------------------------------------------------- cluster */

static size_t orc_find(size_t* parent, size_t i)
{
    while (parent[i] != i) {
        parent[i] = parent[parent[i]]; /* path halving */
        i = parent[i];
    }
    return i;
}

/* The root of every set is its smallest member: the larger root is always
 * hung under the smaller one. */
static void orc_union(size_t* parent, size_t a, size_t b)
{
    size_t ra = orc_find(parent, a), rb = orc_find(parent, b);
    if (ra == rb) return;
    if (ra < rb) parent[rb] = ra; else parent[ra] = rb;
}

typedef struct {
    const uint32_t* shot;
    const uint64_t* toa;
} orc_sort_ctx;
static orc_sort_ctx g_ctx;

static int orc_cmp_shot_toa(const void* a, const void* b)
{
    size_t i = *(const size_t*)a, j = *(const size_t*)b;
    if (g_ctx.shot[i] != g_ctx.shot[j]) return g_ctx.shot[i] < g_ctx.shot[j] ? -1 : 1;
    if (g_ctx.toa[i] != g_ctx.toa[j]) return g_ctx.toa[i] < g_ctx.toa[j] ? -1 : 1;
    return i < j ? -1 : (i > j);
}

static uint32_t orc_absdiff(uint32_t a, uint32_t b) { return a > b ? a - b : b - a; }

/* Step 4.  labels[i] = smallest index j reachable from i. */
int orc_cluster(size_t n, const uint16_t* x, const uint16_t* y,
                const uint32_t* shot, const uint64_t* toa, uint32_t dxy,
                uint32_t dt_ticks, uint64_t* labels, size_t* n_clusters)
{
    size_t* parent = (size_t*)malloc((n ? n : 1) * sizeof(size_t));
    size_t* ord = (size_t*)malloc((n ? n : 1) * sizeof(size_t));
    if (!parent || !ord) { free(parent); free(ord); return ORC_ENOMEM; }
    for (size_t i = 0; i < n; ++i) { parent[i] = i; ord[i] = i; }
    g_ctx.shot = shot;
    g_ctx.toa = toa;
    qsort(ord, n, sizeof(size_t), orc_cmp_shot_toa);

    /* every pair within dt of each other inside one shot is visited once:
     * walk forward from a in time order until the gap exceeds dt */
    for (size_t a = 0; a < n; ++a) {
        size_t i = ord[a];
        for (size_t b = a + 1; b < n; ++b) {
            size_t j = ord[b];
            if (shot[j] != shot[i] || toa[j] - toa[i] > dt_ticks) break;
            if (orc_absdiff(x[i], x[j]) <= dxy && orc_absdiff(y[i], y[j]) <= dxy)
                orc_union(parent, i, j);
        }
    }
    size_t nc = 0;
    for (size_t i = 0; i < n; ++i) {
        labels[i] = orc_find(parent, i);
        if (labels[i] == i) nc++;
    }
    *n_clusters = nc;
    free(parent);
    free(ord);
    return ORC_OK;
}

/* -------------------------------------------------------------- centroid */

static const uint32_t* g_root_shot;
static int orc_cmp_root(const void* a, const void* b)
{
    size_t i = *(const size_t*)a, j = *(const size_t*)b;
    if (g_root_shot[i] != g_root_shot[j]) return g_root_shot[i] < g_root_shot[j] ? -1 : 1;
    return i < j ? -1 : (i > j);
}

/* Step 5.  Hits in (shot, label) order.  ToF of a pixel = toa - trig[shot]. */
int orc_centroid(size_t n, const uint16_t* x, const uint16_t* y,
                 const uint16_t* tot, const uint32_t* shot, const uint64_t* toa,
                 const uint64_t* labels, const uint64_t* trig, size_t n_trig,
                 const double* walk_ns, orc_hit* hits, size_t hit_cap,
                 size_t* n_hits)
{
    *n_hits = 0;
    for (size_t i = 0; i < n; ++i) {
        uint64_t r = labels[i];
        if (r >= n || labels[r] != r || shot[r] != shot[i] || shot[i] >= n_trig)
            return ORC_EINVAL;
    }
    int64_t* W = (int64_t*)calloc(n ? n : 1, sizeof(int64_t));
    int64_t* Sx = (int64_t*)calloc(n ? n : 1, sizeof(int64_t));
    int64_t* Sy = (int64_t*)calloc(n ? n : 1, sizeof(int64_t));
    int64_t* St = (int64_t*)calloc(n ? n : 1, sizeof(int64_t));
    int64_t* Ux = (int64_t*)calloc(n ? n : 1, sizeof(int64_t));
    int64_t* Uy = (int64_t*)calloc(n ? n : 1, sizeof(int64_t));
    int64_t* Ut = (int64_t*)calloc(n ? n : 1, sizeof(int64_t));
    double* Sw = (double*)calloc(n ? n : 1, sizeof(double));
    double* Uw = (double*)calloc(n ? n : 1, sizeof(double));
    uint64_t* cnt = (uint64_t*)calloc(n ? n : 1, sizeof(uint64_t));
    uint64_t* tmin = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    size_t* roots = (size_t*)malloc((n ? n : 1) * sizeof(size_t));
    int rc = ORC_OK;
    if (!W || !Sx || !Sy || !St || !Ux || !Uy || !Ut || !Sw || !Uw || !cnt || !tmin || !roots) {
        rc = ORC_ENOMEM;
        goto done;
    }
    for (size_t i = 0; i < n; ++i) tmin[i] = UINT64_MAX;
    for (size_t i = 0; i < n; ++i) {
        size_t r = (size_t)labels[i];
        int64_t tof = (int64_t)(toa[i] - trig[shot[i]]);
        W[r] += tot[i];
        Sx[r] += (int64_t)tot[i] * x[i];
        Sy[r] += (int64_t)tot[i] * y[i];
        St[r] += (int64_t)tot[i] * tof;
        Ux[r] += x[i];
        Uy[r] += y[i];
        Ut[r] += tof;
        if (walk_ns) {
            Sw[r] += (double)tot[i] * walk_ns[tot[i] & 1023];
            Uw[r] += walk_ns[tot[i] & 1023];
        }
        cnt[r]++;
        if (toa[i] < tmin[r]) tmin[r] = toa[i];
    }
    size_t nr = 0;
    for (size_t i = 0; i < n; ++i)
        if (labels[i] == i) roots[nr++] = i;
    g_root_shot = shot;
    qsort(roots, nr, sizeof(size_t), orc_cmp_root);
    *n_hits = nr;
    if (nr > hit_cap) { rc = ORC_ECAPACITY; goto done; }
    for (size_t k = 0; k < nr; ++k) {
        size_t r = roots[k];
        orc_hit* h = &hits[k];
        memset(h, 0, sizeof(*h));
        h->shot = shot[r];
        h->label = r;
        h->toa_first = tmin[r];
        h->npix = cnt[r];
        h->tot_sum = (uint64_t)W[r];
        if (W[r] > 0) {
            h->x = (double)Sx[r] / (double)W[r];
            h->y = (double)Sy[r] / (double)W[r];
            h->tof_ns = (ORC_TICK_NS * (double)St[r] - Sw[r]) / (double)W[r];
        } else { /* no mass at all: plain mean, flagged */
            h->x = (double)Ux[r] / (double)cnt[r];
            h->y = (double)Uy[r] / (double)cnt[r];
            h->tof_ns = (ORC_TICK_NS * (double)Ut[r] - Uw[r]) / (double)cnt[r];
            h->flags |= 1u;
        }
    }
done:
    free(W); free(Sx); free(Sy); free(St); free(Ux); free(Uy); free(Ut);
    free(Sw); free(Uw); free(cnt); free(tmin); free(roots);
    return rc;
}

/* ---------------------------------------------------- paper local maxima */
/* Sec. V, Local Maxima: with M the row-repeated ToT masked by A (Eq. 6), row
 * i of M - M^T has maximum 0 exactly when no neighbour of i carries more ToT
 * (Eq. 7).  The paper breaks ties by adding 0.001 i to the ToT; that is read
 * here as a tie-break by index: i is a local maximum when every neighbour
 * j != i has (ToT_j, j) < (ToT_i, i) lexicographically.  Each local maximum
 * is one hit whose centroid is Eq. (9) over row i of A (its neighbours and
 * itself): X = sum_j A_ij ToT_j x_j / sum_j A_ij ToT_j, same for Y and ToF.
 * Written out per shot by brute force over all pairs of its pixels.  Hits in
 * (shot, index) order; label = index of the local maximum; npix, tot_sum and
 * toa_first describe its row; a row without ToT gives plain means, flag 1. */
static int orc_nb(const uint16_t* x, const uint16_t* y, const uint64_t* toa, size_t i,
                  size_t j, uint32_t r, uint32_t dt)
{
    const int64_t dx = (int64_t)x[i] - x[j], dy = (int64_t)y[i] - y[j];
    const int64_t d = (int64_t)(toa[i] - toa[j]);
    return (dx < 0 ? -dx : dx) <= r && (dy < 0 ? -dy : dy) <= r && (d < 0 ? -d : d) <= dt;
}

int orc_local_maxima(size_t n, const uint16_t* x, const uint16_t* y, const uint16_t* tot,
                     const uint32_t* shot, const uint64_t* toa, uint32_t dxy, uint32_t dt_ticks,
                     const uint64_t* trig, size_t n_trig, const double* walk_ns, orc_hit* hits,
                     size_t hit_cap, size_t* n_hits)
{
    *n_hits = 0;
    for (size_t i = 0; i < n; ++i)
        if (shot[i] >= n_trig) return ORC_EINVAL;
    size_t* idx = (size_t*)malloc((n ? n : 1) * sizeof(size_t));
    if (!idx) return ORC_ENOMEM;
    for (size_t i = 0; i < n; ++i) idx[i] = i;
    g_root_shot = shot;
    qsort(idx, n, sizeof(size_t), orc_cmp_root); /* by (shot, index) */
    size_t nh = 0;
    int rc = ORC_OK;
    for (size_t a = 0; a < n;) {
        size_t b = a;
        while (b < n && shot[idx[b]] == shot[idx[a]]) ++b;
        for (size_t p = a; p < b; ++p) {
            const size_t i = idx[p];
            int is_max = 1;
            for (size_t q = a; q < b && is_max; ++q) {
                const size_t j = idx[q];
                if (j == i || !orc_nb(x, y, toa, i, j, dxy, dt_ticks)) continue;
                if (tot[j] > tot[i] || (tot[j] == tot[i] && j > i)) is_max = 0;
            }
            if (!is_max) continue;
            int64_t W = 0, Sx = 0, Sy = 0, St = 0, Ux = 0, Uy = 0, Ut = 0;
            double Sw = 0, Uw = 0;
            uint64_t cnt = 0, tmin = UINT64_MAX;
            for (size_t q = a; q < b; ++q) {
                const size_t j = idx[q];
                if (j != i && !orc_nb(x, y, toa, i, j, dxy, dt_ticks)) continue;
                const int64_t tof = (int64_t)(toa[j] - trig[shot[j]]);
                W += tot[j];
                Sx += (int64_t)tot[j] * x[j];
                Sy += (int64_t)tot[j] * y[j];
                St += (int64_t)tot[j] * tof;
                Ux += x[j];
                Uy += y[j];
                Ut += tof;
                if (walk_ns) {
                    Sw += (double)tot[j] * walk_ns[tot[j] & 1023];
                    Uw += walk_ns[tot[j] & 1023];
                }
                cnt++;
                if (toa[j] < tmin) tmin = toa[j];
            }
            if (nh < hit_cap) {
                orc_hit* h = &hits[nh];
                memset(h, 0, sizeof(*h));
                h->shot = shot[i];
                h->label = i;
                h->toa_first = tmin;
                h->npix = cnt;
                h->tot_sum = (uint64_t)W;
                if (W > 0) {
                    h->x = (double)Sx / (double)W;
                    h->y = (double)Sy / (double)W;
                    h->tof_ns = (ORC_TICK_NS * (double)St - Sw) / (double)W;
                } else {
                    h->x = (double)Ux / (double)cnt;
                    h->y = (double)Uy / (double)cnt;
                    h->tof_ns = (ORC_TICK_NS * (double)Ut - Uw) / (double)cnt;
                    h->flags |= 1u;
                }
            }
            ++nh;
        }
        a = b;
    }
    *n_hits = nh;
    if (nh > hit_cap) rc = ORC_ECAPACITY;
    free(idx);
    return rc;
}

/* ----------------------------------------------------------- whole path */

/* Steps 1-5 over one whole packet stream.  Hit labels are indices into the
 * stream-ordered list of kept pixels.  Returns the status of the first step
 * that failed; *n_hits holds the number of hits even when hit_cap is short. */
int orc_run(const uint64_t* pk, size_t n, const orc_params* p, orc_hit* hits,
            size_t hit_cap, size_t* n_hits, orc_stats* st)
{
    size_t cap = n ? n : 1;
    uint16_t* ex = (uint16_t*)malloc(cap * sizeof(uint16_t));
    uint16_t* ey = (uint16_t*)malloc(cap * sizeof(uint16_t));
    uint16_t* et = (uint16_t*)malloc(cap * sizeof(uint16_t));
    uint32_t* es = (uint32_t*)malloc(cap * sizeof(uint32_t));
    uint64_t* ea = (uint64_t*)malloc(cap * sizeof(uint64_t));
    uint64_t* tr = (uint64_t*)malloc(cap * sizeof(uint64_t));
    uint64_t* lab = (uint64_t*)malloc(cap * sizeof(uint64_t));
    int rc = ORC_ENOMEM;
    size_t ne = 0, nt = 0, nc = 0;
    *n_hits = 0;
    if (!ex || !ey || !et || !es || !ea || !tr || !lab) goto done;
    rc = orc_decode(pk, n, p, ex, ey, et, es, ea, cap, &ne, tr, cap, &nt, NULL, st);
    if (rc != ORC_OK) goto done;
    rc = orc_cluster(ne, ex, ey, es, ea, p->dxy, p->dt_ticks, lab, &nc);
    if (rc != ORC_OK) goto done;
    rc = orc_centroid(ne, ex, ey, et, es, ea, lab, tr, nt, p->walk_ns, hits,
                      hit_cap, n_hits);
    st->n_hits = *n_hits;
done:
    free(ex); free(ey); free(et); free(es); free(ea); free(tr); free(lab);
    return rc;
}
