// C ABI of libtpx (declared in include/tpx.h).  Argument checks, workspace
// carving, kernel sequencing on the caller's HIP stream, the single read-back
// of device counters per call, and the host side of the streaming state.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tpx_kernels.h"

using namespace tpx;

namespace {

thread_local std::string g_err;

tpx_status fail(tpx_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

}  // namespace

// error text for the other translation units of the library
tpx_status tpx::report(tpx_status st, const char* msg) { return fail(st, "%s", msg); }

namespace {

#define HIPCHK(x)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return fail(TPX_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

constexpr uint32_t kQ = 1024;           // segment stride (events), default
constexpr int kDefaultFused = 1;        // fused-kernel variant of a new stream
// chunks of at most this many tiles take the persistent launch by default:
// measured faster for 2-tile chunks (64 KiB: 0.160 against 0.183 ms per
// call), slower for 31-32 tiles (0.24 against 0.22 ms)
constexpr uint32_t kPersistentTiles = 4;
constexpr float kTuneKeep = 1.03f;      // autotune keeps the current pair unless beaten by 3%
constexpr uint32_t kQMin = 64, kQMax = 4096;  // strides a stream accepts
constexpr uint32_t kQPaper = 512;       // segment stride of the paper mode: a shot of up to
                                        // 1,536 events always fits one 2,048-event segment
constexpr int kStages = 7;              // timed stages of the stream fast path
constexpr uint64_t kMaxEvents = 0xFFFFFFF0ull;
// packets in one decode call: the tile look-back keeps a kept-event count and a
// trigger-table index in 31 bits each
constexpr uint64_t kMaxCallPkts = (1ull << 31) - 16;

uint64_t ntiles_of(uint64_t n) { return (n + kTilePkts - 1) / kTilePkts; }

tpx_status check_params(const tpx_params* p) {
    if (!p) return fail(TPX_EINVAL, "params is NULL");
    if (p->dxy > 7) return fail(TPX_EINVAL, "dxy must be 0..7 (got %u)", p->dxy);
    if (p->dt_ticks > 65535) return fail(TPX_EINVAL, "dt_ticks must be <= 65535");
    if (p->tof_max_ticks == 0 || p->tof_max_ticks >= (1u << 30))
        return fail(TPX_EINVAL, "tof_max_ticks must be in 1..2^30-1");
    if (p->walk_lut_ns && p->tof_max_ticks >= (1u << 24))
        return fail(TPX_EINVAL, "tof_max_ticks must be < 2^24 with a walk table");
    if (p->trig_subtype > 15) return fail(TPX_EINVAL, "trig_subtype is a 4-bit field");
    if (p->jump_ticks == 0 || p->jump_ticks >= kPixPeriod)
        return fail(TPX_EINVAL, "jump_ticks must be in 1..2^34-1");
    if (p->pix_epoch0 < 0 || p->tdc_epoch0 < 0) return fail(TPX_EINVAL, "negative initial epoch");
    return TPX_OK;
}

// bump allocator over a caller workspace (or a sizing pass with base == 0)
struct Carve {
    uintptr_t base, off;
    template <typename T>
    T* take(uint64_t count) {
        off = (off + 255) & ~(uintptr_t)255;
        T* p = (T*)(base + off);
        off += count * sizeof(T);
        return p;
    }
};

struct DecodeWs {
    DevResults* res;
    TileAcc* sums;
    TileAcc* partial;
    TileAcc* blk;
    TileEntry* entries;
    uint64_t* tdc_slot;
    uint64_t* tab;
    uint64_t* lb;
};
DecodeWs carve_decode(Carve& c, uint64_t n) {
    const uint64_t nt = ntiles_of(n) + 1;
    DecodeWs w;
    w.res = c.take<DevResults>(1);
    w.sums = c.take<TileAcc>(nt);
    w.partial = c.take<TileAcc>(nt);
    w.blk = c.take<TileAcc>(2 * tile_scan_blocks(nt) + 2);
    w.entries = c.take<TileEntry>(nt);
    w.tdc_slot = c.take<uint64_t>(nt * kTilePkts);
    w.tab = c.take<uint64_t>(n + 2);
    w.lb = c.take<uint64_t>(nt);
    return w;
}

struct ClusterWs {
    DevResults* res;
    uint32_t *flags, *scan, *block_tmp, *keys, *vals, *keys2, *vals2, *grp_off, *grp_shot;
    uint32_t *seg_lo, *seg_cnt, *seg_off;
    uint64_t* lb;
    uint32_t* big[6];
    uint64_t* acc;
};
ClusterWs carve_cluster(Carve& c, uint64_t m, bool with_acc) {
    ClusterWs w;
    w.res = c.take<DevResults>(1);
    w.flags = c.take<uint32_t>(m + 1);
    w.scan = c.take<uint32_t>(m + 2);
    w.block_tmp = c.take<uint32_t>(1024);
    w.keys = c.take<uint32_t>(m + 1);
    w.vals = c.take<uint32_t>(m + 1);
    w.keys2 = c.take<uint32_t>(m + 1);
    w.vals2 = c.take<uint32_t>(m + 1);
    w.grp_off = c.take<uint32_t>(m + 2);
    w.grp_shot = c.take<uint32_t>(m + 1);
    w.seg_lo = c.take<uint32_t>(m / kQPaper + 4);
    w.seg_cnt = c.take<uint32_t>(m / kQPaper + 4);
    w.seg_off = c.take<uint32_t>(m / kQPaper + 5);
    w.lb = c.take<uint64_t>(m / kQ + 4);
    for (int k = 0; k < 6; ++k) w.big[k] = c.take<uint32_t>(m + 1);
    w.acc = with_acc ? c.take<uint64_t>(10 * (m + 1)) : nullptr;
    return w;
}

void zero_res(DevResults* r, hipStream_t s) {
    launch_fill_u64((uint64_t*)r, 0, sizeof(DevResults) / 8, s);
}

tpx_status read_res(DevResults* dev, DevResults* host, hipStream_t s) {
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) return fail(TPX_EHIP, "kernel launch failed: %s", hipGetErrorString(le));
    HIPCHK(hipMemcpyAsync(host, dev, sizeof(DevResults), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return TPX_OK;
}

tpx_status res_error(const DevResults& r) {
    if (r.err & kErrStream)
        return fail(TPX_ESTREAM, "triggers go back in time or a wrap count became negative");
    if (r.err & kErrInput) return fail(TPX_EINVAL, "malformed values in an input buffer");
    if (r.err & kErrSpin) return fail(TPX_EINTERNAL, "a look-back wait exceeded its bound");
    if (r.err & kErrCapacity)
        return fail(TPX_ECAPACITY, "open shots hold more events than the carry capacity");
    if (r.err & (kErrLoopFind | kErrLoopUnite | kErrLoopChain))
        return fail(TPX_EINTERNAL, "cluster walk bound exceeded (mask 0x%llx)", r.err);
    if (r.err) return fail(TPX_EINTERNAL, "device error mask 0x%llx", r.err);
    return TPX_OK;
}

void fill_stats(tpx_stats* st, const DevResults& r, uint64_t n_pkts, uint64_t n_events,
                uint64_t n_hits) {
    if (!st) return;
    st->n_packets = n_pkts;
    st->n_pixels = r.n_pixels;
    st->n_tdc = r.n_trig;
    st->n_other = r.n_other;
    st->n_pre_trigger = r.n_pre_trigger;
    st->n_tof_cut = r.n_tof_cut;
    st->n_events = n_events;
    st->n_hits = n_hits;
    st->n_pix_wraps = r.n_pix_wraps;
    st->n_pix_backjumps = r.n_pix_backjumps;
    st->n_tdc_wraps = r.n_tdc_wraps;
    st->n_tdc_backjumps = r.n_tdc_backjumps;
    st->n_late_drop = r.n_late_drop;
}

RunSum run_of(uint32_t has, uint64_t last) {
    return has ? RunSum{last, last, 0, 1} : run_empty();
}

int bits_for(uint64_t max_key) {
    int b = 0;
    while (b < 32 && (max_key >> b)) ++b;
    return b;
}

// the front end shared by tpx_decode and the stream: tiles -> tile state ->
// trigger table (written at tab + n_win)
void launch_front(const uint64_t* pk, uint64_t n, const tpx_params& p, const DecodeWs& w,
                  RunSum pix0, RunSum tdc0, int64_t pe0, int64_t te0, uint64_t* tab,
                  uint64_t n_win, hipStream_t s) {
    const uint64_t nt = ntiles_of(n);
    launch_tile_summary(pk, n, p.trig_subtype, p.jump_ticks, w.sums, w.tdc_slot, s);
    launch_tile_scan(w.sums, nt, TileAcc{pix0, tdc0, 0}, pe0, te0, p.jump_ticks, w.partial, w.blk,
                     w.res, s);
    launch_trig_unwrap(w.sums, w.partial, w.blk, w.tdc_slot, nt, pe0, te0, p.jump_ticks,
                       w.entries, tab + n_win, w.res, s);
    launch_fill_u64(w.lb, 0, nt + 1, s);
}

}  // namespace

// ====================================================================== ABI
// ------------------------------------------------- allocation-free clustering
// tpx_cluster_static's workspace: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  In host code
// the array's name is not a device address: the address is taken once per
// device with hipGetSymbolAddress and only that address is used.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // per device: the address of `scratch`, or null

// The current device's copy of `scratch` (looked up on the first call on
// that device); null with the error reported.
void* scratch_of_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        report(TPX_EHIP, "no current HIP device (or more devices than the library tracks)");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            report(TPX_EHIP, "hipGetSymbolAddress of the static workspace failed");
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

void tpx_params_default(tpx_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->dxy = 1;
    p->dt_ticks = 128;
    p->tof_max_ticks = 64000;
    p->trig_subtype = 0xF;
    p->jump_ticks = 12800000000ull;
    p->pix_epoch0 = 0;
    p->tdc_epoch0 = 0;
    p->close_slack_ticks = 64000;
    p->walk_lut_ns = nullptr;
}

void tpx_unwrap_state_init(tpx_unwrap_state* st, const tpx_params* p) {
    if (!st) return;
    std::memset(st, 0, sizeof *st);
    if (p) {
        st->pix_epoch = p->pix_epoch0;
        st->tdc_epoch = p->tdc_epoch0;
    }
}

const char* tpx_status_str(tpx_status st) {
    switch (st) {
        case TPX_OK: return "ok";
        case TPX_EINVAL: return "invalid argument";
        case TPX_ECAPACITY: return "output capacity too small";
        case TPX_ESTREAM: return "inconsistent stream";
        case TPX_EHIP: return "HIP runtime error";
        case TPX_ENOMEM: return "out of device memory";
        case TPX_EINTERNAL: return "internal error";
        default: return "unknown status";
    }
}

const char* tpx_last_error(void) { return g_err.c_str(); }

size_t tpx_workspace_bytes(size_t max_packets, size_t max_events) {
    Carve a{0, 0};
    carve_decode(a, max_packets);
    Carve b{0, 0};
    carve_cluster(b, max_events, true);
    return (size_t)(std::max(a.off, b.off) + 256);
}

tpx_status tpx_decode(const uint64_t* pkts, size_t n_pkts, const tpx_params* p_h,
                      tpx_unwrap_state* st_h, tpx_events ev, size_t ev_cap, uint64_t* trig_toa,
                      size_t trig_cap, size_t* n_ev_h, size_t* n_trig_h, tpx_stats* stats_h,
                      void* ws, size_t ws_bytes, void* stream) {
    tpx_status rc = check_params(p_h);
    if (rc) return rc;
    if (!st_h || !n_ev_h || !n_trig_h) return fail(TPX_EINVAL, "NULL state or count pointer");
    if (n_pkts && !pkts) return fail(TPX_EINVAL, "pkts is NULL");
    if (ev_cap && (!ev.x || !ev.y || !ev.tot || !ev.shot || !ev.toa))
        return fail(TPX_EINVAL, "an event array is NULL");
    if (trig_cap && !trig_toa) return fail(TPX_EINVAL, "trig_toa is NULL");
    if (n_pkts >= kMaxCallPkts) return fail(TPX_EINVAL, "too many packets in one call");
    if (!ws || ws_bytes < tpx_workspace_bytes(n_pkts, 0))
        return fail(TPX_EINVAL, "workspace too small (need %zu bytes)", tpx_workspace_bytes(n_pkts, 0));
    if (st_h->pix_epoch < 0 || st_h->tdc_epoch < 0) return fail(TPX_EINVAL, "negative epoch in state");
    hipStream_t s = (hipStream_t)stream;
    Carve c{(uintptr_t)ws, 0};
    DecodeWs w = carve_decode(c, n_pkts);
    zero_res(w.res, s);
    const uint64_t n_win = st_h->has_last_trig ? 1 : 0;
    if (n_win) launch_fill_u64(w.tab, st_h->last_trig_toa, 1, s);
    launch_front(pkts, n_pkts, *p_h, w, run_of(st_h->pix_has_last, st_h->pix_last_raw),
                 run_of(st_h->tdc_has_last, st_h->tdc_last_raw), st_h->pix_epoch, st_h->tdc_epoch,
                 w.tab, n_win, s);
    AssignArgs a{};
    a.pk = pkts;
    a.n = n_pkts;
    a.sub = p_h->trig_subtype;
    a.tof_max = p_h->tof_max_ticks;
    a.jump = p_h->jump_ticks;
    a.entries = w.entries;
    a.sums = w.sums;
    a.tab = w.tab;
    a.n_win = n_win;
    a.n_trig_dev = &w.res->n_trig;
    a.first_open = 0;
    a.tab_has_before = st_h->trig_base > n_win;
    a.ev_cap = ev_cap;
    a.soa = ev;
    a.shot_base = st_h->trig_base - n_win;
    a.lb_status = w.lb;
    a.res = w.res;
    launch_assign(a, true, s);
    DevResults r;
    rc = read_res(w.res, &r, s);
    if (rc) return rc;
    *n_ev_h = r.n_kept;
    *n_trig_h = r.n_trig;
    if ((rc = res_error(r))) return rc;
    if (r.n_kept > ev_cap) return fail(TPX_ECAPACITY, "need %llu event slots", r.n_kept);
    if (r.n_trig > trig_cap) return fail(TPX_ECAPACITY, "need %llu trigger slots", r.n_trig);
    if (r.n_trig) {
        HIPCHK(hipMemcpyAsync(trig_toa, w.tab + n_win, r.n_trig * 8, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(&st_h->last_trig_toa, w.tab + n_win + r.n_trig - 1, 8,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        st_h->has_last_trig = 1;
    }
    st_h->pix_epoch = r.pix_epoch_end;
    st_h->tdc_epoch = r.tdc_epoch_end;
    st_h->pix_last_raw = r.pix_last_end;
    st_h->tdc_last_raw = r.tdc_last_end;
    st_h->pix_has_last = (uint32_t)r.pix_has_end;
    st_h->tdc_has_last = (uint32_t)r.tdc_has_end;
    st_h->trig_base += r.n_trig;
    fill_stats(stats_h, r, n_pkts, r.n_kept, 0);
    return TPX_OK;
}

tpx_status tpx_cluster(tpx_events ev, size_t n_ev, const tpx_params* p_h, uint32_t* labels,
                       size_t* n_clusters_h, void* ws, size_t ws_bytes, void* stream) {
    tpx_status rc = check_params(p_h);
    if (rc) return rc;
    if (n_ev >= kMaxEvents) return fail(TPX_EINVAL, "too many events");
    if (n_ev && (!ev.x || !ev.y || !ev.shot || !ev.toa || !ev.tot || !labels))
        return fail(TPX_EINVAL, "an event or label array is NULL");
    if (!ws || ws_bytes < tpx_workspace_bytes(0, n_ev))
        return fail(TPX_EINVAL, "workspace too small (need %zu bytes)", tpx_workspace_bytes(0, n_ev));
    if (n_ev == 0) {
        if (n_clusters_h) *n_clusters_h = 0;
        return TPX_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    Carve c{(uintptr_t)ws, 0};
    ClusterWs w = carve_cluster(c, n_ev, false);
    zero_res(w.res, s);
    launch_fill_u64((uint64_t*)&w.res->n_in, n_ev, 1, s);
    launch_check_events(ev, n_ev, w.res, s);
    DevResults r;
    if ((rc = read_res(w.res, &r, s))) return rc;
    if ((rc = res_error(r))) return rc;
    const uint32_t* sorted_key = ev.shot;
    const uint32_t* perm = nullptr;
    if (r.unsorted) {
        launch_iota_u32(w.vals, n_ev, s);
        HIPCHK(hipMemcpyAsync(w.keys, ev.shot, n_ev * 4, hipMemcpyDeviceToDevice, s));
        uint32_t *ko, *vo;
        radix_sort_pairs(w.keys, w.vals, w.keys2, w.vals2, w.flags, w.scan, w.block_tmp, n_ev,
                         bits_for(r.max_key), s, &ko, &vo);
        sorted_key = ko;
        perm = vo;
    }
    launch_boundaries(sorted_key, n_ev, w.flags, w.scan, w.block_tmp, w.grp_off, w.grp_shot, w.res, s);
    ClusterArgs a{};
    a.soa = ev;
    a.perm = perm;
    a.grp_off = w.grp_off;
    a.grp_shot = w.grp_shot;
    a.n_ev_dev = &w.res->n_in;
    a.n_grp_dev = &w.res->n_groups;
    a.seg_lo = w.seg_lo;
    a.q = kQ;
    a.dxy = p_h->dxy;
    a.dt = p_h->dt_ticks;
    a.labels = labels;
    a.res = w.res;
    a.g_parent = w.big[0];
    a.g_chain = w.big[1];
    a.g_next = w.big[2];
    a.g_t = w.big[3];
    a.g_sl = w.big[4];
    a.g_xy = w.big[5];
    launch_seg_table(w.grp_off, a.n_grp_dev, a.n_ev_dev, nullptr, kQ, n_ev, w.seg_lo, w.res, s);
    launch_cluster(a, true, cluster_grid(n_ev, kQ), s);
    if ((rc = read_res(w.res, &r, s))) return rc;
    if ((rc = res_error(r))) return rc;
    if (n_clusters_h) *n_clusters_h = r.n_hits;
    return TPX_OK;
}

size_t tpx_cluster_static_max_events(void) {
    // largest n whose workspace fits the static array (the workspace grows
    // monotonically with n): bisection over the sizing pass
    size_t lo = 0, hi = kScratchBytes;
    while (lo < hi) {
        const size_t mid = lo + (hi - lo + 1) / 2;
        if (tpx_workspace_bytes(0, mid) <= kScratchBytes) lo = mid; else hi = mid - 1;
    }
    return lo;
}

tpx_status tpx_cluster_static(tpx_events ev, size_t n_ev, const tpx_params* p_h, uint32_t* labels,
                              size_t* n_clusters_h, void* stream) {
    const size_t need = tpx_workspace_bytes(0, n_ev);
    if (need > kScratchBytes)
        return fail(TPX_EINVAL, "%zu events need %zu bytes of workspace; the static workspace "
                    "holds %zu (at most %zu events)", n_ev, need, kScratchBytes,
                    tpx_cluster_static_max_events());
    void* ws = scratch_of_current_device();
    if (!ws) return TPX_EHIP;
    // every buffer of the workspace that must start at zero is cleared by a
    // kernel inside tpx_cluster (no memset nodes, no allocation)
    return tpx_cluster(ev, n_ev, p_h, labels, n_clusters_h, ws, kScratchBytes, stream);
}

tpx_status tpx_local_maxima(tpx_events ev, size_t n_ev, const uint64_t* trig_toa, size_t n_trig,
                            const tpx_params* p_h, tpx_hit* hits, size_t hit_cap,
                            size_t* n_hits_h, void* ws, size_t ws_bytes, void* stream) {
    tpx_status rc = check_params(p_h);
    if (rc) return rc;
    if (!n_hits_h) return fail(TPX_EINVAL, "n_hits_h is NULL");
    if (n_ev >= kMaxEvents) return fail(TPX_EINVAL, "too many events");
    if (n_ev && (!ev.x || !ev.y || !ev.shot || !ev.toa || !ev.tot || !trig_toa))
        return fail(TPX_EINVAL, "an input array is NULL");
    if (hit_cap && !hits) return fail(TPX_EINVAL, "hits is NULL");
    if (!ws || ws_bytes < tpx_workspace_bytes(0, n_ev))
        return fail(TPX_EINVAL, "workspace too small (need %zu bytes)", tpx_workspace_bytes(0, n_ev));
    *n_hits_h = 0;
    if (n_ev == 0) return TPX_OK;
    hipStream_t s = (hipStream_t)stream;
    Carve c{(uintptr_t)ws, 0};
    ClusterWs w = carve_cluster(c, n_ev, false);
    zero_res(w.res, s);
    launch_fill_u64((uint64_t*)&w.res->n_in, n_ev, 1, s);
    launch_check_events(ev, n_ev, w.res, s);
    DevResults r;
    if ((rc = read_res(w.res, &r, s))) return rc;
    if ((rc = res_error(r))) return rc;
    if (r.max_key >= n_trig) return fail(TPX_EINVAL, "shot %llu has no trigger time", r.max_key);
    const uint32_t* sorted_key = ev.shot;
    const uint32_t* perm = nullptr;
    if (r.unsorted) {
        launch_iota_u32(w.vals, n_ev, s);
        HIPCHK(hipMemcpyAsync(w.keys, ev.shot, n_ev * 4, hipMemcpyDeviceToDevice, s));
        uint32_t *ko, *vo;
        radix_sort_pairs(w.keys, w.vals, w.keys2, w.vals2, w.flags, w.scan, w.block_tmp, n_ev,
                         bits_for(r.max_key), s, &ko, &vo);
        sorted_key = ko;
        perm = vo;
    }
    launch_boundaries(sorted_key, n_ev, w.flags, w.scan, w.block_tmp, w.grp_off, w.grp_shot, w.res, s);
    ClusterArgs a{};
    a.soa = ev;
    a.perm = perm;
    a.grp_off = w.grp_off;
    a.grp_shot = w.grp_shot;
    a.n_ev_dev = &w.res->n_in;
    a.n_grp_dev = &w.res->n_groups;
    a.seg_lo = w.seg_lo;
    a.seg_cnt = w.seg_cnt;
    a.seg_off = w.seg_off;
    a.q = kQPaper;
    a.dxy = p_h->dxy;
    a.dt = p_h->dt_ticks;
    a.walk = p_h->walk_lut_ns;
    a.hits = hits;
    a.hit_cap = hit_cap;
    a.res = w.res;
    // per-event scratch of groups too large for LDS
    a.g_parent = w.big[0];
    a.g_next = w.big[2];
    a.g_t = w.big[3];
    a.g_sl = w.big[4];
    a.g_xy = w.big[5];
    launch_seg_table(w.grp_off, a.n_grp_dev, a.n_ev_dev, nullptr, kQPaper, n_ev, w.seg_lo, w.res,
                     s);
    const uint64_t grid = cluster_grid(n_ev, kQPaper);
    launch_paper(a, trig_toa, false, grid, s);
    launch_scan_u32(w.seg_cnt, w.seg_off, 0, &w.res->n_seg, w.block_tmp, s);
    launch_paper(a, trig_toa, true, grid, s);
    if ((rc = read_res(w.res, &r, s))) return rc;
    if ((rc = res_error(r))) return rc;
    *n_hits_h = r.n_hits;
    if (r.n_hits > hit_cap) return fail(TPX_ECAPACITY, "need %llu hit slots", r.n_hits);
    return TPX_OK;
}

tpx_status tpx_centroid(tpx_events ev, const uint32_t* labels, size_t n_ev,
                        const uint64_t* trig_toa, size_t n_trig, const tpx_params* p_h,
                        tpx_hit* hits, size_t hit_cap, size_t* n_hits_h, void* ws,
                        size_t ws_bytes, void* stream) {
    tpx_status rc = check_params(p_h);
    if (rc) return rc;
    if (!n_hits_h) return fail(TPX_EINVAL, "n_hits_h is NULL");
    if (n_ev >= kMaxEvents) return fail(TPX_EINVAL, "too many events");
    if (n_ev && (!ev.x || !ev.y || !ev.shot || !ev.toa || !ev.tot || !labels || !trig_toa))
        return fail(TPX_EINVAL, "an input array is NULL");
    if (hit_cap && !hits) return fail(TPX_EINVAL, "hits is NULL");
    if (!ws || ws_bytes < tpx_workspace_bytes(0, n_ev))
        return fail(TPX_EINVAL, "workspace too small (need %zu bytes)", tpx_workspace_bytes(0, n_ev));
    *n_hits_h = 0;
    if (n_ev == 0) return TPX_OK;
    hipStream_t s = (hipStream_t)stream;
    Carve c{(uintptr_t)ws, 0};
    ClusterWs w = carve_cluster(c, n_ev, true);
    zero_res(w.res, s);
    launch_check_events(ev, n_ev, w.res, s);
    launch_cent_init(w.acc, n_ev, s);
    launch_cent_accum(ev, labels, n_ev, trig_toa, n_trig, p_h->walk_lut_ns, w.acc, w.res, s);
    launch_root_flags(labels, n_ev, w.flags, s);
    launch_scan_u32(w.flags, w.scan, n_ev, nullptr, w.block_tmp, s);
    launch_compact_roots(w.flags, w.scan, n_ev, w.keys2, s);
    DevResults r;
    uint32_t n_roots = 0;
    HIPCHK(hipMemcpyAsync(&n_roots, w.scan + n_ev, 4, hipMemcpyDeviceToHost, s));
    if ((rc = read_res(w.res, &r, s))) return rc;
    if ((rc = res_error(r))) return rc;
    *n_hits_h = n_roots;
    if (n_roots > hit_cap) return fail(TPX_ECAPACITY, "need %u hit slots", n_roots);
    const uint32_t* order = w.keys2;
    if (r.unsorted) {
        launch_gather_keys(ev.shot, w.keys2, w.keys, n_roots, s);
        HIPCHK(hipMemcpyAsync(w.vals, w.keys2, (size_t)n_roots * 4, hipMemcpyDeviceToDevice, s));
        uint32_t *ko, *vo;
        radix_sort_pairs(w.keys, w.vals, w.grp_off, w.grp_shot, w.flags, w.scan, w.block_tmp,
                         n_roots, bits_for(r.max_key), s, &ko, &vo);
        order = vo;
    }
    launch_cent_emit(ev, order, n_roots, w.acc, trig_toa, p_h->walk_lut_ns, hits, hit_cap, s);
    HIPCHK(hipStreamSynchronize(s));
    return TPX_OK;
}

}  // extern "C"

// ==================================================================== stream
struct tpx_stream {
    tpx_params p;
    uint64_t max_chunk;
    uint64_t tab_cap, ev_cap, carry_cap, seg_cap;
    std::vector<void*> allocs;
    uint64_t device_bytes = 0;  // sum of the allocations
    DevResults* res;
    DevResults* res_h;
    DecodeWs dw;
    uint64_t* tab[2];
    uint32_t *shot_cnt, *shot_off;
    uint64_t* ev;
    uint64_t* c_ev[2];
    uint32_t* c_shot[2];
    uint64_t* c_gidx[2];
    // general path
    uint32_t *shot_arr, *keys, *vals, *keys2, *vals2, *flags, *scan, *grp_off, *grp_shot;
    uint64_t* ev_sorted;
    uint32_t* block_tmp;
    uint32_t *seg_lo, *seg_cnt, *seg_off, *rank;
    uint32_t* big[6];
    uint64_t* g_acc;
    tpx_hit* hits_tmp;      // staged hits of the fused kernel
    // staged assignment: kept events (and shots) per tile, per-tile records
    uint64_t* ev_stage;
    uint32_t *shot_stage, *tile_cnt, *tile_lo, *tile_hi, *tile_off;
    unsigned long long* tile_stat;
    uint32_t* hit_index;    // hit of every event of the last call (when kept)
    uint32_t* defer;        // routed kernel: segments left to its persistent launch
    uint32_t n_cu;          // compute units of the device (persistent grid)
    unsigned int* qs;       // work-queue counters of the persistent chunk kernel
    ChunkArgs* chunk_args;  // its arguments: device copy
    ChunkArgs* chunk_args_h;  // and the pinned host block they are copied from
    uint32_t persistent;    // chunks of at most this many tiles in one persistent launch
    // committed host state
    int64_t pix_epoch, tdc_epoch;
    uint64_t pix_last, tdc_last;
    uint32_t pix_has, tdc_has;
    uint64_t win_base;      // global trigger index of tab[cur][0]
    uint64_t n_win;         // window triggers at tab[cur][0..n_win)
    uint64_t first_open;    // window index of the first open shot
    uint64_t max_t_plus1;
    uint64_t ev_next;       // global index of the next kept event
    uint64_t n_carry;       // events of open shots in c_*[cur]
    uint32_t carry_rebase;  // subtract from c_shot[cur] to get window indices
    uint64_t carry_last1;   // window index of the last carried event + 1 (0 = none)
    int cur;
    uint32_t q;             // segment stride of the clustering (events)
    int kernel;             // fused-kernel variant, or -1: staged cluster + centroid kernels
    int keep_hit_index;     // record the hit of every event (tpx_stream_patches)
    int last_fused;         // the last call took the fused kernel
    // the last successful call's clustering (its events, ranks and segment
    // offsets stay in place until the next call): patches of its hits
    ClusterArgs last_c;
    uint64_t last_grid, last_hits;
    int last_ok;
    uint64_t n_fallback;    // chunks that needed the general (sorting) path
    // optional per-stage timing with HIP events on the caller's stream
    int timing;
    hipEvent_t tev[kStages + 1];
    float stage_ms[kStages];
};

namespace {

template <typename T>
tpx_status dalloc(tpx_stream* s, T** p, uint64_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<uint64_t>(count, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TPX_ENOMEM, "hipMalloc of %llu bytes failed",
                    (unsigned long long)(count * sizeof(T)));
    }
    s->allocs.push_back(q);
    s->device_bytes += std::max<uint64_t>(count, 1) * sizeof(T);
    *p = (T*)q;
    return TPX_OK;
}

void free_stream(tpx_stream* s) {
    if (s->timing)
        for (auto& e : s->tev) (void)hipEventDestroy(e);
    for (void* q : s->allocs) (void)hipFree(q);
    if (s->res_h) (void)hipHostFree(s->res_h);
    if (s->chunk_args_h) (void)hipHostFree(s->chunk_args_h);
    delete s;
}

void mark(tpx_stream* s, int i, hipStream_t hs) {
    if (s->timing) (void)hipEventRecord(s->tev[i], hs);
}

// shot assignment of the chunk's pixels: tiles into their staging ranges,
// a prefix sum of the tiles' counts, then every kept event to
// ev[n_carry + its position] (and its shot to shot_final when given)
void stream_assign(tpx_stream* s, AssignArgs a, uint32_t* shot_final, hipStream_t hs) {
    const uint64_t nt = ntiles_of(a.n);
    a.ev = s->ev_stage;
    a.ev_off = 0;
    a.ev_cap = nt * kTilePkts;
    a.shot_out = shot_final ? s->shot_stage : nullptr;
    a.tile_cnt = s->tile_cnt;
    a.tile_lo = s->tile_lo;
    a.tile_hi = s->tile_hi;
    a.tile_stat = s->tile_stat;
    launch_assign_staged(a, hs);
    launch_scan_u32(s->tile_cnt, s->tile_off, nt, nullptr, s->block_tmp, hs);
    launch_assign_place(a, s->tile_off, s->ev, s->n_carry, s->ev_cap, shot_final, hs);
}

ClusterArgs stream_cluster_args(tpx_stream* s, tpx_hit* hits, uint64_t hit_cap) {
    ClusterArgs a{};
    a.q = s->q;
    a.dxy = s->p.dxy;
    a.dt = s->p.dt_ticks;
    a.carry_gidx = s->c_gidx[s->cur];
    a.n_carry = s->n_carry;
    a.ev_base = s->ev_next;
    a.tab = s->tab[s->cur];
    a.tab_base = s->win_base;
    a.walk = s->p.walk_lut_ns;
    a.hits = hits;
    a.hit_cap = hit_cap;
    a.rank = s->rank;
    a.seg_cnt = s->seg_cnt;
    a.seg_off = s->seg_off;
    a.res = s->res;
    a.g_parent = s->big[0];
    a.g_chain = s->big[1];
    a.g_next = s->big[2];
    a.g_t = s->big[3];
    a.g_sl = s->big[4];
    a.g_xy = s->big[5];
    a.g_acc = s->g_acc;
    a.hits_tmp = s->hits_tmp;
    a.hit_index = s->keep_hit_index ? s->hit_index : nullptr;
    return a;
}

// fused kernel for radius 1 (times of flight in 16 bits) unless the staged
// kernels were asked for
bool use_fused(const tpx_stream* s) {
    return s->p.dxy == 1 && s->p.tof_max_ticks < 65536 && s->kernel >= 0;
}

// components and hits of the closed events: one fused launch, or the staged
// cluster -> prefix -> centroid kernels
void stream_cluster(tpx_stream* s, const ClusterArgs& c, uint64_t grid, hipStream_t hs) {
    s->last_c = c;
    s->last_grid = grid;
    s->last_fused = use_fused(s);
    if (s->last_fused) {
        mark(s, 4, hs);
        launch_cluster_fused(c, grid, s->kernel, s->defer, s->n_cu, hs);
        mark(s, 5, hs);
        launch_scan_u32(s->seg_cnt, s->seg_off, 0, &s->res->n_seg, s->block_tmp, hs);
        launch_hit_compact(c, grid, hs);
        mark(s, 6, hs);
        return;
    }
    mark(s, 4, hs);
    launch_cluster(c, false, grid, hs);
    mark(s, 5, hs);
    launch_scan_u32(s->seg_cnt, s->seg_off, 0, &s->res->n_seg, s->block_tmp, hs);
    launch_seg_centroid(c, grid, hs);
    mark(s, 6, hs);
}

AssignArgs stream_assign_args(tpx_stream* s, const uint64_t* chunk, uint64_t n) {
    AssignArgs a{};
    a.pk = chunk;
    a.n = n;
    a.sub = s->p.trig_subtype;
    a.tof_max = s->p.tof_max_ticks;
    a.jump = s->p.jump_ticks;
    a.entries = s->dw.entries;
    a.sums = s->dw.sums;
    a.tab = s->tab[s->cur];
    a.n_win = s->n_win;
    a.n_trig_dev = &s->res->n_trig;
    a.first_open = s->first_open;
    a.tab_has_before = s->win_base > 0;
    a.ev = s->ev;
    a.ev_off = s->n_carry;
    a.ev_cap = s->ev_cap;
    a.carry_last1 = s->carry_last1;
    a.lb_status = s->dw.lb;
    a.res = s->res;
    return a;
}


// decode front end of one chunk (shared by both paths)
void stream_front(tpx_stream* s, const uint64_t* chunk, uint64_t n, hipStream_t hs) {
    zero_res(s->res, hs);
    mark(s, 0, hs);
    const uint64_t nt = ntiles_of(n);
    launch_tile_summary(chunk, n, s->p.trig_subtype, s->p.jump_ticks, s->dw.sums, s->dw.tdc_slot,
                        hs);
    mark(s, 1, hs);
    launch_tile_scan(s->dw.sums, nt,
                     TileAcc{run_of(s->pix_has, s->pix_last), run_of(s->tdc_has, s->tdc_last), 0},
                     s->pix_epoch, s->tdc_epoch, s->p.jump_ticks, s->dw.partial, s->dw.blk, s->res,
                     hs);
    launch_trig_unwrap(s->dw.sums, s->dw.partial, s->dw.blk, s->dw.tdc_slot, nt, s->pix_epoch,
                       s->tdc_epoch, s->p.jump_ticks, s->dw.entries, s->tab[s->cur] + s->n_win,
                       s->res, hs);
    launch_fill_u64(s->dw.lb, 0, nt + 1, hs);
}

// The fast path of a chunk of at most chunk_max_tiles() tiles in one
// persistent launch (k_stream_chunk): the same steps and buffers as the
// separate launches below; the stage clock shows the launch as the cluster
// stage.
tpx_status stream_persistent(tpx_stream* s, const uint64_t* chunk, uint64_t n, int flush,
                             tpx_hit* hits, uint64_t hit_cap, hipStream_t hs) {
    const uint64_t nt = ntiles_of(n);
    for (int i = 0; i <= 4; ++i) mark(s, i, hs);
    ChunkArgs p{};
    AssignArgs a = stream_assign_args(s, chunk, n);
    a.shot_cnt = s->shot_cnt;
    a.ev = s->ev_stage;  // staged per tile, as stream_assign
    a.ev_off = 0;
    a.ev_cap = nt * kTilePkts;
    a.shot_out = nullptr;
    a.tile_cnt = s->tile_cnt;
    a.tile_lo = s->tile_lo;
    a.tile_hi = s->tile_hi;
    a.tile_stat = s->tile_stat;
    p.a = a;
    ClusterArgs c = stream_cluster_args(s, hits, hit_cap);
    c.ev = s->ev;
    c.grp_off = s->shot_off;
    c.n_ev_dev = &s->res->n_close_ev;
    c.n_grp_dev = &s->res->n_close_grp;
    c.skip = &s->res->unsorted;
    c.seg_lo = s->seg_lo;
    p.c = c;
    p.sums = s->dw.sums;
    p.tdc_slot = s->dw.tdc_slot;
    p.entries = s->dw.entries;
    p.tab_new = s->tab[s->cur] + s->n_win;
    p.init = TileAcc{run_of(s->pix_has, s->pix_last), run_of(s->tdc_has, s->tdc_last), 0};
    p.pe0 = s->pix_epoch;
    p.te0 = s->tdc_epoch;
    p.tile_off = s->tile_off;
    p.ev = s->ev;
    p.ev_cap = s->ev_cap;
    p.c_ev_in = s->c_ev[s->cur];
    p.c_shot_in = s->c_shot[s->cur];
    p.n_carry = s->n_carry;
    p.carry_rebase = s->carry_rebase;
    p.flush = flush;
    p.max_t_plus1_prev = s->max_t_plus1;
    p.slack = s->p.close_slack_ticks;
    const int nx = 1 - s->cur;
    p.c_gidx_in = s->c_gidx[s->cur];
    p.c_ev_out = s->c_ev[nx];
    p.c_shot_out = s->c_shot[nx];
    p.c_gidx_out = s->c_gidx[nx];
    p.carry_cap = s->carry_cap;
    p.qs = s->qs;
    p.ntiles = (uint32_t)nt;
    p.seg_grid = (uint32_t)cluster_grid(s->n_carry + n, s->q);
    s->last_c = c;
    s->last_grid = p.seg_grid;
    s->last_fused = 1;
    // the previous call synchronised the stream: the host block is free
    *s->chunk_args_h = p;
    if (hipMemcpyAsync(s->chunk_args, s->chunk_args_h, sizeof(ChunkArgs), hipMemcpyHostToDevice,
                       hs) != hipSuccess)
        return fail(TPX_EHIP, "argument copy failed");
    launch_stream_chunk(p, s->chunk_args, s->n_cu, hs);
    for (int i = 5; i <= 7; ++i) mark(s, i, hs);
    tpx_status rc = read_res(s->res, s->res_h, hs);
    if (rc == TPX_OK && s->timing)
        for (int i = 0; i < kStages; ++i)
            (void)hipEventElapsedTime(&s->stage_ms[i], s->tev[i], s->tev[i + 1]);
    return rc;
}

tpx_status stream_fast(tpx_stream* s, const uint64_t* chunk, uint64_t n, int flush, tpx_hit* hits,
                       uint64_t hit_cap, hipStream_t hs) {
    if (ntiles_of(n) <= s->persistent && use_fused(s))
        return stream_persistent(s, chunk, n, flush, hits, hit_cap, hs);
    stream_front(s, chunk, n, hs);
    const uint64_t rows = s->n_win + n + 1;  // bound of the table rows (window + new triggers)
    launch_fill_u32_dev(s->shot_cnt, 0, s->n_win, &s->res->n_trig, 2, hs);
    launch_carry_in(s->c_ev[s->cur], s->c_shot[s->cur], s->n_carry, s->carry_rebase, s->ev, nullptr,
                    s->shot_cnt, hs);
    AssignArgs a = stream_assign_args(s, chunk, n);
    a.shot_cnt = s->shot_cnt;
    mark(s, 2, hs);
    stream_assign(s, a, nullptr, hs);
    mark(s, 3, hs);
    launch_set_rows(s->res, s->n_win, hs);
    launch_scan_u32(s->shot_cnt, s->shot_off, 0, &s->res->n_groups, s->block_tmp, hs);
    launch_close(s->tab[s->cur], &s->res->n_trig, s->n_win, s->first_open, flush, s->max_t_plus1,
                 s->p.tof_max_ticks, s->p.close_slack_ticks, s->shot_off, s->res, hs);
    ClusterArgs c = stream_cluster_args(s, hits, hit_cap);
    c.ev = s->ev;
    c.grp_off = s->shot_off;
    c.n_ev_dev = &s->res->n_close_ev;
    c.n_grp_dev = &s->res->n_close_grp;
    c.skip = &s->res->unsorted;
    c.seg_lo = s->seg_lo;
    launch_seg_table(c.grp_off, c.n_grp_dev, c.n_ev_dev, c.skip, s->q, rows, s->seg_lo, s->res, hs);
    stream_cluster(s, c, cluster_grid(s->n_carry + n, s->q), hs);
    const int nx = 1 - s->cur;
    launch_carry_out(s->ev, nullptr, nullptr, s->shot_off, &s->res->n_groups, &s->res->n_close_ev,
                     &s->res->n_kept, s->c_gidx[s->cur], s->n_carry, s->ev_next, s->c_ev[nx],
                     s->c_shot[nx], s->c_gidx[nx], s->carry_cap, s->res, hs);
    mark(s, 7, hs);
    tpx_status rc = read_res(s->res, s->res_h, hs);
    if (rc == TPX_OK && s->timing)
        for (int i = 0; i < kStages; ++i)
            (void)hipEventElapsedTime(&s->stage_ms[i], s->tev[i], s->tev[i + 1]);
    return rc;
}

// Events not in shot order: materialise every event's shot, sort stably by
// shot, and cluster through the permutation.
tpx_status stream_general(tpx_stream* s, const uint64_t* chunk, uint64_t n, int flush,
                          tpx_hit* hits, uint64_t hit_cap, uint64_t n_kept, uint64_t n_trig,
                          hipStream_t hs) {
    stream_front(s, chunk, n, hs);
    launch_carry_in(s->c_ev[s->cur], s->c_shot[s->cur], s->n_carry, s->carry_rebase, s->ev,
                    s->shot_arr, nullptr, hs);
    AssignArgs a = stream_assign_args(s, chunk, n);
    stream_assign(s, a, s->shot_arr, hs);
    const uint64_t N = s->n_carry + n_kept;
    const uint64_t n_tab = s->n_win + n_trig;
    HIPCHK(hipMemcpyAsync(s->keys, s->shot_arr, N * 4, hipMemcpyDeviceToDevice, hs));
    launch_iota_u32(s->vals, N, hs);
    uint32_t *ko, *vo;
    radix_sort_pairs(s->keys, s->vals, s->keys2, s->vals2, s->flags, s->scan, s->block_tmp, N,
                     bits_for(n_tab ? n_tab - 1 : 0), hs, &ko, &vo);
    launch_gather_packed(s->ev, vo, s->ev_sorted, N, hs);
    launch_close(s->tab[s->cur], &s->res->n_trig, s->n_win, s->first_open, flush, s->max_t_plus1,
                 s->p.tof_max_ticks, s->p.close_slack_ticks, nullptr, s->res, hs);
    launch_boundaries(ko, N, s->flags, s->scan, s->block_tmp, s->grp_off, s->grp_shot, s->res, hs);
    launch_close_sorted(ko, N, s->grp_shot, s->res, hs);
    ClusterArgs c = stream_cluster_args(s, hits, hit_cap);
    c.ev = s->ev_sorted;
    c.perm = vo;
    c.grp_off = s->grp_off;
    c.grp_shot = s->grp_shot;
    c.n_ev_dev = &s->res->n_close_ev;
    c.n_grp_dev = &s->res->n_close_list;
    c.seg_lo = s->seg_lo;
    launch_seg_table(c.grp_off, c.n_grp_dev, c.n_ev_dev, nullptr, s->q, N, s->seg_lo, s->res, hs);
    stream_cluster(s, c, cluster_grid(N, s->q), hs);
    const int nx = 1 - s->cur;
    launch_carry_out(s->ev_sorted, vo, ko, nullptr, nullptr, &s->res->n_close_ev, &s->res->n_kept,
                     s->c_gidx[s->cur], s->n_carry, s->ev_next, s->c_ev[nx], s->c_shot[nx],
                     s->c_gidx[nx], s->carry_cap, s->res, hs);
    return read_res(s->res, s->res_h, hs);
}

}  // namespace

extern "C" {

tpx_status tpx_stream_create(const tpx_params* p_h, size_t max_chunk_pkts, tpx_stream** out_h) {
    tpx_status rc = check_params(p_h);
    if (rc) return rc;
    if (!out_h) return fail(TPX_EINVAL, "out_h is NULL");
    if (max_chunk_pkts == 0 || max_chunk_pkts >= kMaxCallPkts / 2)
        return fail(TPX_EINVAL, "max_chunk_pkts out of range");
    tpx_stream* s = new tpx_stream();  // value-initialised: every scalar starts at zero
    s->p = *p_h;
    s->max_chunk = max_chunk_pkts;
    const uint64_t n = max_chunk_pkts;
    s->carry_cap = n;
    s->ev_cap = n + s->carry_cap;
    s->tab_cap = n + s->carry_cap + 2;
    s->q = kQ;
    s->kernel = kDefaultFused;
    s->persistent = kPersistentTiles;
    s->seg_cap = s->ev_cap / kQMin + 4;
    if (hipHostMalloc((void**)&s->res_h, sizeof(DevResults), 0) != hipSuccess) {
        (void)hipGetLastError();
        s->res_h = nullptr;
        free_stream(s);
        return fail(TPX_ENOMEM, "pinned host allocation failed");
    }
    const uint64_t nt = ntiles_of(n) + 1;
#define ALLOC(ptr, count)                                   \
    if ((rc = dalloc(s, &(ptr), (count))) != TPX_OK) {      \
        free_stream(s);                                     \
        return rc;                                          \
    }
    ALLOC(s->res, 1);
    s->dw.res = s->res;
    ALLOC(s->dw.sums, nt);
    ALLOC(s->dw.partial, nt);
    ALLOC(s->dw.blk, 2 * tile_scan_blocks(nt) + 2);
    ALLOC(s->dw.entries, nt);
    ALLOC(s->dw.tdc_slot, nt * kTilePkts);
    ALLOC(s->dw.lb, nt + 1);
    ALLOC(s->tab[0], s->tab_cap);
    ALLOC(s->tab[1], s->tab_cap);
    ALLOC(s->shot_cnt, s->tab_cap + 2);
    ALLOC(s->shot_off, s->tab_cap + 2);
    ALLOC(s->ev, s->ev_cap);
    ALLOC(s->ev_stage, nt * kTilePkts);
    ALLOC(s->shot_stage, nt * kTilePkts);
    ALLOC(s->tile_cnt, nt);
    ALLOC(s->tile_lo, nt);
    ALLOC(s->tile_hi, nt);
    ALLOC(s->tile_off, nt + 2);
    ALLOC(s->tile_stat, 8 * nt);
    for (int k = 0; k < 2; ++k) {
        ALLOC(s->c_ev[k], s->carry_cap);
        ALLOC(s->c_shot[k], s->carry_cap);
        ALLOC(s->c_gidx[k], s->carry_cap);
    }
    ALLOC(s->shot_arr, s->ev_cap);
    ALLOC(s->keys, s->ev_cap);
    ALLOC(s->vals, s->ev_cap);
    ALLOC(s->keys2, s->ev_cap);
    ALLOC(s->vals2, s->ev_cap);
    ALLOC(s->flags, s->ev_cap + 1);
    ALLOC(s->scan, s->ev_cap + 2);
    ALLOC(s->grp_off, s->ev_cap + 2);
    ALLOC(s->grp_shot, s->ev_cap + 1);
    ALLOC(s->ev_sorted, s->ev_cap);
    ALLOC(s->block_tmp, 1024);
    ALLOC(s->seg_lo, s->seg_cap);
    ALLOC(s->seg_cnt, s->seg_cap);
    ALLOC(s->seg_off, s->seg_cap + 1);
    ALLOC(s->rank, s->ev_cap);
    for (int k = 0; k < 6; ++k) ALLOC(s->big[k], s->ev_cap);
    ALLOC(s->g_acc, 8 * s->ev_cap);
    ALLOC(s->hits_tmp, s->ev_cap);
    ALLOC(s->hit_index, s->ev_cap);
    ALLOC(s->defer, s->seg_cap);
    ALLOC(s->qs, chunk_queue_words());
    ALLOC(s->chunk_args, 1);
    if (hipHostMalloc((void**)&s->chunk_args_h, sizeof(ChunkArgs), 0) != hipSuccess) {
        (void)hipGetLastError();
        s->chunk_args_h = nullptr;
        free_stream(s);
        return fail(TPX_ENOMEM, "pinned host allocation failed");
    }
#undef ALLOC
    launch_fill_u32(s->qs, 0, chunk_queue_words(), nullptr);
    if (hipStreamSynchronize(nullptr) != hipSuccess) {
        (void)hipGetLastError();
        free_stream(s);
        return fail(TPX_EHIP, "clearing the stream's counters failed");
    }
    {
        int dev = 0, cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cu <= 0) {
            (void)hipGetLastError();
            cu = 256;
        }
        s->n_cu = (uint32_t)cu;
    }
    s->pix_epoch = p_h->pix_epoch0;
    s->tdc_epoch = p_h->tdc_epoch0;
    *out_h = s;
    return TPX_OK;
}

void tpx_stream_destroy(tpx_stream* s) {
    if (s) free_stream(s);
}

tpx_status tpx_process_stream(tpx_stream* s, const uint64_t* chunk, size_t n_pkts, int flush,
                              tpx_hit* hits, size_t hit_cap, size_t* n_hits_h, tpx_stats* stats_h,
                              void* stream) {
    if (!s) return fail(TPX_EINVAL, "stream is NULL");
    if (!n_hits_h) return fail(TPX_EINVAL, "n_hits_h is NULL");
    if (n_pkts > s->max_chunk) return fail(TPX_EINVAL, "chunk larger than max_chunk_pkts");
    if (n_pkts && !chunk) return fail(TPX_EINVAL, "chunk is NULL");
    if (hit_cap && !hits) return fail(TPX_EINVAL, "hits is NULL");
    if (s->n_win + n_pkts + 2 > s->tab_cap) return fail(TPX_EINTERNAL, "trigger window overflow");
    hipStream_t hs = (hipStream_t)stream;
    s->last_ok = 0;
    tpx_status rc = stream_fast(s, chunk, n_pkts, flush, hits, hit_cap, hs);
    if (rc) return rc;
    DevResults r = *s->res_h;
    *n_hits_h = 0;
    if (r.unsorted && !(r.err & kErrStream)) {
        // the decode is repeated bit for bit; only the grouping changes
        const uint64_t n_kept = r.n_kept, n_trig = r.n_trig;
        rc = stream_general(s, chunk, n_pkts, flush, hits, hit_cap, n_kept, n_trig, hs);
        if (rc) return rc;
        r = *s->res_h;
        s->n_fallback++;
    }
    if ((rc = res_error(r))) return rc;
    *n_hits_h = r.n_hits;
    if (r.n_hits > hit_cap) return fail(TPX_ECAPACITY, "need %llu hit slots", r.n_hits);

    // commit: next window starts at the last closed shot (kept for the cut of
    // late pixels), carried events move to the other buffer
    const uint64_t n_tab = s->n_win + r.n_trig;
    const uint64_t s_close = r.n_close_grp;
    const uint64_t ws = s_close > 0 ? s_close - 1 : 0;
    const int nx = 1 - s->cur;
    if (n_tab > ws) {
        HIPCHK(hipMemcpyAsync(s->tab[nx], s->tab[s->cur] + ws, (n_tab - ws) * 8,
                              hipMemcpyDeviceToDevice, hs));
    }
    uint64_t last_trig = 0;
    if (r.n_trig)
        HIPCHK(hipMemcpyAsync(&last_trig, s->tab[s->cur] + n_tab - 1, 8, hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    s->pix_epoch = r.pix_epoch_end;
    s->tdc_epoch = r.tdc_epoch_end;
    s->pix_last = r.pix_last_end;
    s->tdc_last = r.tdc_last_end;
    s->pix_has = (uint32_t)r.pix_has_end;
    s->tdc_has = (uint32_t)r.tdc_has_end;
    s->win_base += ws;
    s->n_win = n_tab - ws;
    s->first_open = s_close - ws;
    s->max_t_plus1 = std::max<uint64_t>(s->max_t_plus1, r.max_t_plus1);
    if (r.n_trig) s->max_t_plus1 = std::max<uint64_t>(s->max_t_plus1, last_trig + 1);
    s->ev_next += r.n_kept;
    s->n_carry = s->n_carry + r.n_kept - r.n_close_ev;
    s->carry_rebase = (uint32_t)ws;
    s->carry_last1 = s->n_carry ? (r.carry_last - ws) : 0;
    s->cur = nx;
    s->last_hits = r.n_hits;
    s->last_ok = 1;
    fill_stats(stats_h, r, n_pkts, r.n_kept, r.n_hits);
    return TPX_OK;
}

// checkpoint layout: header, window triggers, carried events
struct StreamCkpt {
    uint64_t magic, version;
    tpx_params p;
    int64_t pix_epoch, tdc_epoch;
    uint64_t pix_last, tdc_last, pix_has, tdc_has;
    uint64_t win_base, n_win, first_open, max_t_plus1, ev_next, n_carry, carry_last1;
};
constexpr uint64_t kCkptMagic = 0x7470785354524d31ull;  // "tpxSTRM1"

tpx_status tpx_stream_get_state(const tpx_stream* s, void* buf_h, size_t* bytes_h) {
    if (!s || !bytes_h) return fail(TPX_EINVAL, "NULL argument");
    const size_t need = sizeof(StreamCkpt) + s->n_win * 8 + s->n_carry * (8 + 4 + 8);
    if (!buf_h) {
        *bytes_h = need;
        return TPX_OK;
    }
    if (*bytes_h < need) {
        *bytes_h = need;
        return fail(TPX_ECAPACITY, "state needs %zu bytes", need);
    }
    StreamCkpt h{};
    h.magic = kCkptMagic;
    h.version = 1;
    h.p = s->p;
    h.p.walk_lut_ns = nullptr;
    h.pix_epoch = s->pix_epoch;
    h.tdc_epoch = s->tdc_epoch;
    h.pix_last = s->pix_last;
    h.tdc_last = s->tdc_last;
    h.pix_has = s->pix_has;
    h.tdc_has = s->tdc_has;
    h.win_base = s->win_base;
    h.n_win = s->n_win;
    h.first_open = s->first_open;
    h.max_t_plus1 = s->max_t_plus1;
    h.ev_next = s->ev_next;
    h.n_carry = s->n_carry;
    h.carry_last1 = s->carry_last1;
    uint8_t* b = (uint8_t*)buf_h;
    std::memcpy(b, &h, sizeof h);
    b += sizeof h;
    HIPCHK(hipMemcpy(b, s->tab[s->cur], s->n_win * 8, hipMemcpyDeviceToHost));
    b += s->n_win * 8;
    HIPCHK(hipMemcpy(b, s->c_ev[s->cur], s->n_carry * 8, hipMemcpyDeviceToHost));
    b += s->n_carry * 8;
    std::vector<uint32_t> sh(s->n_carry);
    HIPCHK(hipMemcpy(sh.data(), s->c_shot[s->cur], s->n_carry * 4, hipMemcpyDeviceToHost));
    for (auto& v : sh) v -= s->carry_rebase;
    std::memcpy(b, sh.data(), s->n_carry * 4);
    b += s->n_carry * 4;
    HIPCHK(hipMemcpy(b, s->c_gidx[s->cur], s->n_carry * 8, hipMemcpyDeviceToHost));
    *bytes_h = need;
    return TPX_OK;
}

tpx_status tpx_stream_set_state(tpx_stream* s, const void* buf_h, size_t bytes) {
    if (s) s->last_ok = 0;
    if (!s || !buf_h) return fail(TPX_EINVAL, "NULL argument");
    if (bytes < sizeof(StreamCkpt)) return fail(TPX_EINVAL, "state buffer too short");
    StreamCkpt h;
    std::memcpy(&h, buf_h, sizeof h);
    if (h.magic != kCkptMagic || h.version != 1) return fail(TPX_EINVAL, "not a stream state");
    const size_t need = sizeof(StreamCkpt) + h.n_win * 8 + h.n_carry * (8 + 4 + 8);
    if (bytes < need) return fail(TPX_EINVAL, "state buffer too short");
    if (h.n_win + 2 > s->tab_cap || h.n_carry > s->carry_cap)
        return fail(TPX_ECAPACITY, "state does not fit this stream's capacity");
    if (h.p.dxy != s->p.dxy || h.p.dt_ticks != s->p.dt_ticks ||
        h.p.tof_max_ticks != s->p.tof_max_ticks || h.p.trig_subtype != s->p.trig_subtype ||
        h.p.jump_ticks != s->p.jump_ticks)
        return fail(TPX_EINVAL, "state was saved with different parameters");
    const uint8_t* b = (const uint8_t*)buf_h + sizeof h;
    const int c = s->cur;
    HIPCHK(hipMemcpy(s->tab[c], b, h.n_win * 8, hipMemcpyHostToDevice));
    b += h.n_win * 8;
    HIPCHK(hipMemcpy(s->c_ev[c], b, h.n_carry * 8, hipMemcpyHostToDevice));
    b += h.n_carry * 8;
    HIPCHK(hipMemcpy(s->c_shot[c], b, h.n_carry * 4, hipMemcpyHostToDevice));
    b += h.n_carry * 4;
    HIPCHK(hipMemcpy(s->c_gidx[c], b, h.n_carry * 8, hipMemcpyHostToDevice));
    s->pix_epoch = h.pix_epoch;
    s->tdc_epoch = h.tdc_epoch;
    s->pix_last = h.pix_last;
    s->tdc_last = h.tdc_last;
    s->pix_has = (uint32_t)h.pix_has;
    s->tdc_has = (uint32_t)h.tdc_has;
    s->win_base = h.win_base;
    s->n_win = h.n_win;
    s->first_open = h.first_open;
    s->max_t_plus1 = h.max_t_plus1;
    s->ev_next = h.ev_next;
    s->n_carry = h.n_carry;
    s->carry_rebase = 0;
    s->carry_last1 = h.carry_last1;
    return TPX_OK;
}

// Diagnostics for tests and benchmarks: chunks that took the general path.
uint64_t tpx_stream_fallback_count(const tpx_stream* s) { return s ? s->n_fallback : 0; }

static const char* const kStageNames[kStages] = {"tile_summary", "tile_prefix", "assign", "group",
                                                 "cluster",      "centroid",    "carry"};

tpx_status tpx_stream_set_timing(tpx_stream* s, int enable) {
    if (!s) return fail(TPX_EINVAL, "stream is NULL");
    if (enable && !s->timing) {
        for (auto& e : s->tev) HIPCHK(hipEventCreate(&e));
        s->timing = 1;
    } else if (!enable && s->timing) {
        for (auto& e : s->tev) (void)hipEventDestroy(e);
        s->timing = 0;
    }
    return TPX_OK;
}

tpx_status tpx_stream_get_timing(const tpx_stream* s, float* ms_h, size_t n, size_t* n_stages_h) {
    if (!s || !n_stages_h) return fail(TPX_EINVAL, "NULL argument");
    *n_stages_h = kStages;
    if (!s->timing) return fail(TPX_EINVAL, "timing is not enabled");
    for (size_t i = 0; i < n && i < (size_t)kStages; ++i) ms_h[i] = s->stage_ms[i];
    return TPX_OK;
}

const char* tpx_stream_stage_name(size_t i) { return i < (size_t)kStages ? kStageNames[i] : ""; }

tpx_status tpx_stream_set_segment(tpx_stream* s, uint32_t q) {
    if (!s) return fail(TPX_EINVAL, "stream is NULL");
    if (q < kQMin || q > kQMax)
        return fail(TPX_EINVAL, "segment stride %u outside [%u, %u]", q, kQMin, kQMax);
    s->q = q;
    return TPX_OK;
}

uint32_t tpx_stream_get_segment(const tpx_stream* s) { return s ? s->q : 0; }

size_t tpx_stream_device_bytes(const tpx_stream* s) { return s ? (size_t)s->device_bytes : 0; }

int tpx_stream_kernel_count(void) { return fused_variants(); }

const char* tpx_stream_kernel_name(int k) {
    return k < 0 ? "staged cluster and centroid kernels" : fused_variant_name(k);
}

tpx_status tpx_stream_set_kernel(tpx_stream* s, int k) {
    if (!s) return fail(TPX_EINVAL, "stream is NULL");
    if (k < -1 || k >= fused_variants())
        return fail(TPX_EINVAL, "kernel %d outside [-1, %d)", k, fused_variants());
    s->kernel = k;
    return TPX_OK;
}

int tpx_stream_get_kernel(const tpx_stream* s) { return s ? s->kernel : -2; }

tpx_status tpx_stream_set_persistent(tpx_stream* s, int max_tiles) {
    if (!s) return fail(TPX_EINVAL, "stream is NULL");
    if (max_tiles < 0 || (uint32_t)max_tiles > chunk_max_tiles())
        return fail(TPX_EINVAL, "max_tiles %d outside [0, %u]", max_tiles, chunk_max_tiles());
    s->persistent = (uint32_t)max_tiles;
    return TPX_OK;
}

int tpx_stream_get_persistent(const tpx_stream* s) { return s ? (int)s->persistent : -1; }

tpx_status tpx_stream_set_patches(tpx_stream* s, int enable) {
    if (!s) return fail(TPX_EINVAL, "stream is NULL");
    s->keep_hit_index = enable ? 1 : 0;
    s->last_ok = 0;  // the last call's events carry no hit index yet
    return TPX_OK;
}

size_t tpx_stream_patch_workspace_bytes(size_t n_hits) { return n_hits * 99 * 4 + 256; }

tpx_status tpx_stream_patches(tpx_stream* s, const tpx_hit* hits, size_t n_hits, uint16_t* feat,
                              void* ws, size_t ws_bytes, void* stream) {
    if (!s) return fail(TPX_EINVAL, "stream is NULL");
    if (!s->last_ok) return fail(TPX_EINVAL, "no completed tpx_process_stream call to take hits from");
    if (n_hits != s->last_hits)
        return fail(TPX_EINVAL, "n_hits (%zu) is not the last call's hit count (%llu)", n_hits,
                    (unsigned long long)s->last_hits);
    if (n_hits && (!hits || !feat)) return fail(TPX_EINVAL, "hits or feat is NULL");
    if (!ws || ws_bytes < tpx_stream_patch_workspace_bytes(n_hits))
        return fail(TPX_EINVAL, "workspace too small");
    if (s->last_fused && !s->keep_hit_index)
        return fail(TPX_EINVAL, "tpx_stream_set_patches(s, 1) must precede the call whose hits "
                    "are patched");
    if (n_hits == 0) return TPX_OK;
    hipStream_t hs = (hipStream_t)stream;
    int* err = (int*)((char*)ws + n_hits * 99 * 4);
    launch_stream_patches(s->last_c, s->last_grid, s->last_fused, hits, n_hits, (uint32_t*)ws,
                          feat, err, hs);
    int e = 0;
    HIPCHK(hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    if (e) return fail(TPX_EINTERNAL, "an event's component has no hit of the last call");
    return TPX_OK;
}

// Times the chunk at every candidate stride (best of `reps`, HIP events on
// the call's stream), restoring the stream state before every run; keeps the
// fastest stride and leaves the stream state as it was.
tpx_status tpx_stream_autotune(tpx_stream* s, const uint64_t* chunk, size_t n_pkts, int flush,
                               tpx_hit* hits, size_t hit_cap, const uint32_t* cand_h,
                               size_t n_cand, const int* kern_h, size_t n_kern, int reps,
                               float* ms_h, uint32_t* best_h, int* best_kern_h, void* stream) {
    if (!s || !cand_h || !best_h) return fail(TPX_EINVAL, "NULL argument");
    if (n_cand == 0 || reps < 1) return fail(TPX_EINVAL, "no candidates or repetitions");
    for (size_t i = 0; i < n_cand; ++i)
        if (cand_h[i] < kQMin || cand_h[i] > kQMax)
            return fail(TPX_EINVAL, "segment stride %u outside [%u, %u]", cand_h[i], kQMin, kQMax);
    const int k_now = s->kernel;
    const size_t nk = kern_h ? n_kern : 1;
    if (nk == 0) return fail(TPX_EINVAL, "no kernel candidates");
    for (size_t j = 0; kern_h && j < nk; ++j)
        if (kern_h[j] < -1 || kern_h[j] >= fused_variants())
            return fail(TPX_EINVAL, "kernel %d outside [-1, %d)", kern_h[j], fused_variants());
    size_t bytes = 0;
    tpx_status rc = tpx_stream_get_state(s, nullptr, &bytes);
    if (rc) return rc;
    std::vector<uint8_t> saved(bytes);
    if ((rc = tpx_stream_get_state(s, saved.data(), &bytes))) return rc;
    const uint32_t q0 = s->q;
    const uint64_t fb0 = s->n_fallback;
    hipStream_t hs = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(TPX_EHIP, "event creation failed");
    }
    float best = 3.0e38f, t_now = -1.f;
    uint32_t best_q = q0;
    int best_k = k_now;
    for (size_t j = 0; j < nk && rc == TPX_OK; ++j) {
        s->kernel = kern_h ? kern_h[j] : k_now;
        for (size_t i = 0; i < n_cand && rc == TPX_OK; ++i) {
            s->q = cand_h[i];
            float t_min = 3.0e38f;
            for (int r = 0; r < reps && rc == TPX_OK; ++r) {
                if ((rc = tpx_stream_set_state(s, saved.data(), bytes))) break;
                size_t nh = 0;
                float ms = 0.f;
                if (hipEventRecord(e0, hs) != hipSuccess) rc = fail(TPX_EHIP, "event record failed");
                if (!rc) rc = tpx_process_stream(s, chunk, n_pkts, flush, hits, hit_cap, &nh, nullptr,
                                                 stream);
                if (!rc && (hipEventRecord(e1, hs) != hipSuccess ||
                            hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = fail(TPX_EHIP, "event timing failed");
                if (!rc) t_min = std::min(t_min, ms);
            }
            if (ms_h) ms_h[j * n_cand + i] = t_min;
            if (!rc && s->kernel == k_now && cand_h[i] == q0) t_now = t_min;
            if (!rc && t_min < best) {
                best = t_min;
                best_q = cand_h[i];
                best_k = s->kernel;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // a win within the timing noise does not displace the configuration in
    // force, so that repeated tunings of one workload agree
    if (!rc && t_now >= 0.f && t_now <= best * kTuneKeep) {
        best_q = q0;
        best_k = k_now;
    }
    const tpx_status rs = tpx_stream_set_state(s, saved.data(), bytes);
    s->n_fallback = fb0;
    s->q = rc ? q0 : best_q;
    s->kernel = rc ? k_now : best_k;
    if (rc) return rc;
    if (rs) return rs;
    *best_h = best_q;
    if (best_kern_h) *best_kern_h = best_k;
    return TPX_OK;
}

}  // extern "C"
