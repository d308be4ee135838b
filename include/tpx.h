/*
 * tpx.h -- C ABI of the MI355X (gfx950) TimePix3 VMI hot path.
 *
 * The library turns a stream of 64-bit TimePix3 packets into particle hits:
 * it decodes pixel and trigger words, unwraps their counters, assigns each
 * pixel to its laser shot with a time-of-flight cut, groups the pixels of a
 * shot into hits by space-time connectivity and reduces every hit to a
 * ToT-weighted centroid (x, y, ToF).  Method: arXiv 2603.04942, "Fast
 * array-based particle coincidence detection in a TimePix3-based velocity map
 * imaging instrument" (Sec. III data stream, Sec. IV preprocessing, Sec. V
 * centroiding).  Every step runs in HIP kernels on the device.
 *
 * Conventions for every entry point:
 *  - Pointers are HIP device pointers unless the parameter name ends in _h
 *    (host).  The caller owns every buffer; only tpx_stream_create allocates.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    work is ordered on it.  A call that returns a count through a _h pointer
 *    synchronises `stream` before returning (these are the only sync points).
 *  - No exception crosses the ABI.  On error the call returns a negative
 *    status, outputs are unspecified, state objects are left unchanged, and
 *    tpx_last_error() describes the failure.  TPX_ECAPACITY stores the
 *    required element count into the corresponding _h count, so the call can
 *    be retried with a larger buffer.  Argument errors (TPX_EINVAL) are
 *    detected before any kernel is launched; malformed input values inside
 *    device buffers are detected on the device and reported after the sync.
 *  - Times are integer ticks of 1.5625 ns (25/16 ns, i.e. 256 of the chip's
 *    25/4096 ns units, Sec. IV).  ToT is in 25 ns counts.
 *  - Thread safety: distinct tpx_stream objects may be used concurrently from
 *    different host threads on different HIP streams; one object must not be
 *    used by two calls at once.
 */
#ifndef TPX_H
#define TPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tpx_status;
#define TPX_OK 0
#define TPX_EINVAL (-1)    /* bad argument or malformed input values          */
#define TPX_ECAPACITY (-2) /* an output buffer is too small (see _h count)    */
#define TPX_ESTREAM (-3)   /* triggers go back in time, or a wrap count < 0   */
#define TPX_EHIP (-4)      /* a HIP runtime call failed                       */
#define TPX_ENOMEM (-5)    /* device allocation failed (tpx_stream_create)    */
#define TPX_EINTERNAL (-6) /* an internal consistency check failed            */

/* Processing parameters (Sec. IV and Sec. V).  Fill with tpx_params_default
 * and override fields.  Limits are checked on every call (TPX_EINVAL). */
typedef struct {
    uint32_t dxy;           /* spatial radius r of the neighbourhood, Chebyshev
                               distance, inclusive (Eq. 4); 1 = 8-connected.
                               0..7                                            */
    uint32_t dt_ticks;      /* time radius r_t, |dToA| <= dt_ticks (Eq. 4 on
                               the ToF axis); 128 = 200 ns.  0..65535          */
    uint32_t tof_max_ticks; /* keep a pixel when ToF <= this (Sec. IV, 100 us
                               = 64000).  1..2^30-1                            */
    uint32_t trig_subtype;  /* TDC subtype nibble that marks a laser trigger;
                               0xF = TDC1 rising edge                          */
    uint64_t jump_ticks;    /* unwrap threshold (Sec. IV, 20 s = 1.28e10).
                               Must be below both wrap periods                 */
    int64_t pix_epoch0;     /* pixel-counter wraps before the first pixel word */
    int64_t tdc_epoch0;     /* trigger-counter wraps before the first trigger  */
    uint64_t close_slack_ticks; /* streaming: shot s is closed once trigger s+1
                               has been seen and a pixel later than T[s] +
                               tof_max + slack has arrived (default 64000)     */
    const float* walk_lut_ns;   /* NULL, or 1024 device floats Delta ToF(ToT)
                               in ns subtracted from each pixel's ToF before
                               the time centroid (Eq. 1).  Default NULL.       */
} tpx_params;

void tpx_params_default(tpx_params* p_h);

/* Decoded pixel events, structure of arrays (device pointers).  `shot`
 * indexes the trigger table that came with the events; `toa` is the unwrapped
 * arrival tick. */
typedef struct {
    uint16_t* x;   /* 0..255 */
    uint16_t* y;   /* 0..255 */
    uint16_t* tot; /* 0..1023 */
    uint32_t* shot;
    uint64_t* toa;
} tpx_events;

/* One particle hit (Eq. 8-9 over one connected component).  48 bytes. */
typedef struct {
    float x, y;         /* ToT-weighted centroid in pixels (pixel centres at
                           integer coordinates)                               */
    float tof_ns;       /* ToT-weighted mean ToF in ns after the shot trigger */
    uint32_t npix;      /* pixels in the hit                                  */
    uint64_t shot;      /* shot (trigger) index                               */
    uint64_t label;     /* smallest event index in the hit                    */
    uint64_t toa_first; /* earliest unwrapped ToA in the hit, ticks           */
    uint32_t tot_sum;   /* sum of ToT                                          */
    uint32_t flags;     /* bit 0: sum of ToT was 0, plain means were used     */
} tpx_hit;

typedef struct {
    uint64_t n_packets, n_pixels, n_tdc, n_other, n_pre_trigger, n_tof_cut,
        n_events, n_hits, n_pix_wraps, n_pix_backjumps, n_tdc_wraps,
        n_tdc_backjumps, n_late_drop;
} tpx_stats;

/* Unwrap and trigger state carried between tpx_decode calls on consecutive
 * pieces of one stream.  Initialise with tpx_unwrap_state_init. */
typedef struct {
    int64_t pix_epoch, tdc_epoch;  /* wraps in force                          */
    uint64_t pix_last_raw, tdc_last_raw;
    uint32_t pix_has_last, tdc_has_last;
    uint64_t trig_base;            /* global index of the next trigger        */
    uint64_t last_trig_toa;        /* unwrapped time of trigger trig_base-1   */
    uint32_t has_last_trig, pad;
} tpx_unwrap_state;

void tpx_unwrap_state_init(tpx_unwrap_state* st_h, const tpx_params* p_h);

/* Device workspace needed by tpx_decode / tpx_cluster / tpx_centroid /
 * tpx_local_maxima for up to max_packets packets or max_events events.  The
 * workspace holds only transient data; its contents need not be preserved
 * between calls. */
size_t tpx_workspace_bytes(size_t max_packets, size_t max_events);

/* Decode, unwrap and assign (Sec. III; Sec. IV, ToA Unwrapping and
 * Eliminating Background Counts).
 *  pkts[n_pkts]   device, 64-bit words in stream order.
 *  st_h           in: state before pkts[0]; out (on success): after.
 *  ev, ev_cap     kept pixels in stream order; ev.shot = global trigger index
 *                 (st_h->trig_base + k for the k-th trigger of this call, or
 *                 trig_base-1 for pixels after the previous call's last one).
 *  trig_toa       the unwrapped triggers of this call, trig_cap entries.
 *  n_ev_h, n_trig_h, stats_h  host outputs (stats_h may be NULL).
 * Pixels before any trigger are dropped (n_pre_trigger); pixels whose ToF
 * exceeds tof_max_ticks are dropped (n_tof_cut).  TPX_ESTREAM when triggers go
 * back in time or a wrap count would become negative. */
tpx_status tpx_decode(const uint64_t* pkts, size_t n_pkts, const tpx_params* p_h,
                      tpx_unwrap_state* st_h, tpx_events ev, size_t ev_cap,
                      uint64_t* trig_toa, size_t trig_cap, size_t* n_ev_h,
                      size_t* n_trig_h, tpx_stats* stats_h, void* ws,
                      size_t ws_bytes, void* stream);

/* Group events into hits (Sec. V, Neighborhoods, Eqs. 3-5, closed
 * transitively): i and j are connected when ev.shot[i] == ev.shot[j],
 * |x_i - x_j| <= dxy, |y_i - y_j| <= dxy and |toa_i - toa_j| <= dt_ticks.
 * labels[i] = the smallest index j connected to i (events need not be sorted
 * by shot).  n_clusters_h (may be NULL) = number of hits. */
tpx_status tpx_cluster(tpx_events ev, size_t n_ev, const tpx_params* p_h,
                       uint32_t* labels, size_t* n_clusters_h, void* ws,
                       size_t ws_bytes, void* stream);

/* tpx_cluster for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments and results without a workspace argument.  The
 * workspace is a 64 MiB array in the library's own device memory (one per
 * GPU, held until the process ends, its address looked up on the first call
 * on each device); this call makes no hipMalloc, hipFree or other allocating
 * call.  n_ev may be at most tpx_cluster_static_max_events() (493,275
 * events); larger inputs return TPX_EINVAL before any launch.  Every
 * call on one GPU shares that array: calls that overlap on one GPU (two host
 * threads, or two HIP streams without ordering between them) race and must
 * be serialised by the caller.  Synchronises `stream` like tpx_cluster. */
size_t tpx_cluster_static_max_events(void);
tpx_status tpx_cluster_static(tpx_events ev, size_t n_ev, const tpx_params* p_h,
                              uint32_t* labels, size_t* n_clusters_h, void* stream);

/* Walk calibration (Sec. IV, ToT-ToF Correlation Correction, Eq. 1) from the
 * decoded events of a calibration run (one ion species at one true ToF):
 *   1. the pixels of the ion peak: tof_lo <= ToF <= tof_hi (ticks; ToF =
 *      toa - trig_toa[shot]);
 *   2. per ToT value the centre of its ToF distribution: the maximum-
 *      likelihood centre of a Gaussian, i.e. the slice's mean ToF (ns);
 *   3. Eq. (1), <ToF>(ToT) = a / (ToT + b)^d + c, fitted to the centres of
 *      the ToT values with at least min_count pixels by least squares
 *      weighted by their pixel counts (= a fit over the individual pixels;
 *      Levenberg-Marquardt on the host, b kept above -min ToT, d in
 *      [0.05, 8]).
 * params_h (host, 4): a, b, c, d (ns, ToT counts); c is the peak's ToF.
 * count_h (host u32[1024], may be NULL): pixels per ToT value in the window;
 * mean_h (host double[1024], may be NULL): their mean ToF in ns (NaN if none).
 * lut (device float[1024], may be NULL): walk(ToT) = a / (ToT + b)^d in ns
 * (ToT values at or below -b take the value of the smallest one above), the
 * table that tpx_params.walk_lut_ns takes (true ToF = measured - walk).
 * ws: tpx_walk_fit_workspace_bytes() device bytes.  Errors: TPX_EINVAL (NULL
 * pointers, tof_hi < tof_lo, min_count 0, a shot without trigger time, fewer
 * than 4 usable ToT values).  Synchronises the stream. */
size_t tpx_walk_fit_workspace_bytes(void);
tpx_status tpx_walk_fit(tpx_events ev, size_t n_ev, const uint64_t* trig_toa, size_t n_trig,
                        uint64_t tof_lo, uint64_t tof_hi, uint32_t min_count, double* params_h,
                        uint32_t* count_h, double* mean_h, float* lut, void* ws, size_t ws_bytes,
                        void* stream);

/* The paper's own hits (Sec. V, Local Maxima and Centroiding; Eqs. 6-7 and
 * Eq. 9 on A itself), event mode.  Event i is a hit when no neighbour (same
 * shot, |dx| <= dxy, |dy| <= dxy, |ToA difference| <= dt_ticks) carries more
 * ToT; between equal ToT the later event wins (the paper's +0.001 i tie-break,
 * read as a tie-break by index).  Its centroid is Eq. (9) over itself and its
 * direct neighbours (not the transitive closure): x = sum(ToT x) / sum(ToT),
 * the same for y and ToF = ToA - trig_toa[shot] (minus walk_lut_ns[ToT] when
 * given); a row without ToT gives plain means and flag bit 0.
 *   ev, n_ev      device SoA events (any order; shots need not be sorted)
 *   trig_toa      device u64[n_trig], trigger time of every shot value
 *   hits          device tpx_hit[hit_cap], written in (shot, index) order;
 *                 label = event index of the maximum, npix / tot_sum /
 *                 toa_first describe its row
 *   n_hits_h      host: number of hits (also on TPX_ECAPACITY)
 *   ws, ws_bytes  device workspace of at least tpx_workspace_bytes(0, n_ev)
 * Shots of any size: a group of shots larger than the 2,048 events one
 * workgroup holds in LDS keeps its per-event arrays in the workspace.
 * Errors: TPX_EINVAL (NULL pointers, x or y > 255, ToT > 1023, a shot value
 * >= n_trig), TPX_ECAPACITY (hit_cap too small).  Synchronises the stream. */
tpx_status tpx_local_maxima(tpx_events ev, size_t n_ev, const uint64_t* trig_toa, size_t n_trig,
                            const tpx_params* p, tpx_hit* hits, size_t hit_cap, size_t* n_hits_h,
                            void* ws, size_t ws_bytes, void* stream);

/* ToT-weighted centroids (Sec. V, Centroiding, Eqs. 8-9) of the hits given by
 * `labels` (as produced by tpx_cluster: labels[i] is the smallest index of i's
 * hit).  ToF = toa - trig_toa[shot].  Hits come out in (shot, label) order. */
tpx_status tpx_centroid(tpx_events ev, const uint32_t* labels, size_t n_ev,
                        const uint64_t* trig_toa, size_t n_trig,
                        const tpx_params* p_h, tpx_hit* hits, size_t hit_cap,
                        size_t* n_hits_h, void* ws, size_t ws_bytes,
                        void* stream);

/* Streaming: decode -> cluster -> centroid over consecutive chunks of one
 * packet stream, carrying unwrap state and the pixels of shots that are still
 * open across chunk boundaries.  Hit labels are global kept-pixel indices in
 * stream order; hit shots are global trigger indices. */
typedef struct tpx_stream tpx_stream;

/* Allocates device memory for chunks of up to max_chunk_pkts packets. */
tpx_status tpx_stream_create(const tpx_params* p_h, size_t max_chunk_pkts,
                             tpx_stream** out_h);

/* Process one chunk.  Hits of every shot closed by this chunk (all shots when
 * flush != 0) are written in (shot, label) order.  A pixel that belongs to a
 * shot closed by an earlier chunk is counted in n_late_drop. */
tpx_status tpx_process_stream(tpx_stream* s, const uint64_t* chunk,
                              size_t n_pkts, int flush, tpx_hit* hits,
                              size_t hit_cap, size_t* n_hits_h,
                              tpx_stats* stats_h, void* stream);

/* Checkpoint: serialise the stream state (unwrap state, trigger window, open
 * shots' pixels) into a host buffer.  With buf_h == NULL only the size is
 * returned in *bytes_h. */
tpx_status tpx_stream_get_state(const tpx_stream* s, void* buf_h, size_t* bytes_h);
tpx_status tpx_stream_set_state(tpx_stream* s, const void* buf_h, size_t bytes);
void tpx_stream_destroy(tpx_stream* s);

/* Diagnostics: number of chunks of this stream whose kept pixels were not in
 * shot order and took the general (sorting) path. */
uint64_t tpx_stream_fallback_count(const tpx_stream* s);

/* Diagnostics: per-stage device time of the last tpx_process_stream call on
 * the fast path, in ms, measured with HIP events recorded on the call's
 * stream between the stages (tile_summary, tile_prefix, assign, group,
 * cluster, centroid, carry).  Enabling creates the events; timing adds one
 * event record per stage and nothing else. */
tpx_status tpx_stream_set_timing(tpx_stream* s, int enable);
tpx_status tpx_stream_get_timing(const tpx_stream* s, float* ms_h, size_t n,
                                 size_t* n_stages_h);
const char* tpx_stream_stage_name(size_t i);

/* Segment stride of the stream's clustering: consecutive shots are packed
 * into segments that start every q kept events (a segment ends at the end of
 * the shot that crosses the next start), one workgroup per segment; 64 <= q
 * <= 4096, default 1024.  Results do not depend on q, only the time.
 *
 * Kernel of the stream's clustering (radius 1): tpx_stream_kernel_count()
 * variants of the fused segment kernel (components, moments and hits of a
 * segment in one workgroup; they differ in the height of the LDS pixel image
 * and the workgroup size; tpx_stream_kernel_name names them), or -1 for the
 * staged kernels (components, then moments and hits in a second launch).
 * Other radii always take the staged kernels.  Results do not depend on the
 * kernel.  Default 1 (a 256x16 image, 512 threads, eight waves per SIMD).
 *
 * tpx_stream_autotune (the sweep of the uneven-shot workload) runs the chunk
 * at every pair of candidate q (cand_h[n_cand]) and kernel (kern_h[n_kern];
 * NULL = the stream's current kernel only), best of `reps` each, timed with
 * HIP events on `stream`, restoring the stream state before each run and
 * after the last; writes the times to ms_h (host, [n_kern][n_cand], may be
 * NULL) and keeps the fastest pair (*best_h, *best_kern_h, which may be
 * NULL), except that the pair in force when called, if it is a candidate,
 * stays unless the fastest beats it by more than 3%.  hits / hit_cap as in tpx_process_stream; on an error the stream
 * keeps its state, its former q and its former kernel. */
tpx_status tpx_stream_set_segment(tpx_stream* s, uint32_t q);
uint32_t tpx_stream_get_segment(const tpx_stream* s);
/* Device memory the stream holds (sum of its allocations). */
size_t tpx_stream_device_bytes(const tpx_stream* s);
int tpx_stream_kernel_count(void);
const char* tpx_stream_kernel_name(int k);
tpx_status tpx_stream_set_kernel(tpx_stream* s, int k);
int tpx_stream_get_kernel(const tpx_stream* s);
/* Persistent launch of small chunks (batching over triggers, Sec. VI, in one
 * launch): a chunk of at most max_tiles tiles of 4,096 words (0 <= max_tiles
 * <= 512; default 4) that takes the fused clustering kernel runs the whole
 * fast path -- decode, unwrap, shot assignment, grouping, components,
 * moments, hits, carry -- as one launch of a persistent grid whose
 * workgroups take work items (tiles, the prefix over tiles, segments, ...)
 * from a ticket counter in dependency order; inside it, segments are
 * clustered by the 2,048-event configuration of variant 1 whatever the
 * stream's variant (larger segments keep their arrays in global scratch).
 * Results do not depend on the setting.  Larger chunks, the staged kernels
 * and chunks whose events are out of shot order take the separate launches.
 * The stage clock reports such a call's whole launch as its cluster stage.
 * set: TPX_EINVAL outside the range; get returns the limit, or -1 for a
 * NULL stream. */
tpx_status tpx_stream_set_persistent(tpx_stream* s, int max_tiles);
int tpx_stream_get_persistent(const tpx_stream* s);
tpx_status tpx_stream_autotune(tpx_stream* s, const uint64_t* chunk, size_t n_pkts, int flush,
                               tpx_hit* hits, size_t hit_cap, const uint32_t* cand_h,
                               size_t n_cand, const int* kern_h, size_t n_kern, int reps,
                               float* ms_h, uint32_t* best_h, int* best_kern_h, void* stream);

/* Continuous batching over one stream (the streaming workload's chunked
 * acquisition, Sec. IV: the unwrap runs across the whole stream).  Chunks are
 * admitted into a device ring as they arrive; every run processes all whole
 * chunks admitted so far, up to max_batch_pkts packets, as one
 * tpx_process_stream call.  Because the stream path gives the same hits for
 * any split of the stream into chunks, batching changes only when hits
 * appear, never what they are.
 *   tpx_service_create  max_batch_pkts: largest batch (and chunk); ring_pkts
 *                       >= max_batch_pkts: admission capacity.  Allocates the
 *                       ring, a staging buffer and a tpx_stream.
 *   tpx_service_submit  reserves ring space and copies n_pkts words (device
 *                       memory when chunk_on_device, else host) into it on
 *                       the service's own stream, after the work already on
 *                       `stream` (which may still be writing the chunk);
 *                       *seq_h = the chunk's number (0, 1, ...).  TPX_EINVAL
 *                       when n_pkts > max_batch_pkts, TPX_ECAPACITY when the
 *                       ring is full (the words of unprocessed chunks and of
 *                       the batch in flight stay reserved); the service is
 *                       then unchanged.
 *   tpx_service_run     one batch: hits of the shots it closes (all shots when
 *                       flush and the batch holds every admitted chunk) as in
 *                       tpx_process_stream; *n_done_h = chunks processed so
 *                       far.  With nothing admitted it still flushes; with
 *                       no chunk ready and no flush it returns at once (no
 *                       hits, nothing launched).  On an
 *                       error the batch stays admitted.  The batch's copies
 *                       are waited for on the device.  Synchronises `stream`.
 * One host thread may submit while another runs: the admission copies of new
 * chunks then overlap the batch on the GPU.  Apart from that pair, calls on
 * one service must not overlap. */
typedef struct tpx_service tpx_service;
tpx_status tpx_service_create(const tpx_params* p_h, size_t max_batch_pkts, size_t ring_pkts,
                              tpx_service** out_h);
tpx_status tpx_service_submit(tpx_service* sv, const uint64_t* chunk, size_t n_pkts,
                              int chunk_on_device, uint64_t* seq_h, void* stream);
tpx_status tpx_service_run(tpx_service* sv, int flush, tpx_hit* hits, size_t hit_cap,
                           size_t* n_hits_h, uint64_t* n_done_h, tpx_stats* stats_h,
                           void* stream);
void tpx_service_destroy(tpx_service* sv);
/*   tpx_service_device_bytes  device memory the service holds (its stream,
 *                       ring and staging buffer).
 *   tpx_service_set_segment  segment stride of the service's stream (as
 *                       tpx_stream_set_segment); not while a run is on the GPU.
 *   tpx_service_replay  paced replay with a native producer thread: chunk k
 *                       (chunk words of the device-resident stream pk[n]) is
 *                       submitted when its last word would have been acquired
 *                       at pkts_per_s packets per second; the calling thread
 *                       runs the service whenever admitted chunks are ready
 *                       (their copies enqueued; flush with the last).  lat_ms_h[k] (host, may be NULL) =
 *                       completion of the run that processed chunk k minus
 *                       its release; *n_chunks_h chunks, *n_runs_h runs.  The
 *                       service must hold no unprocessed chunks.  hits /
 *                       hit_cap receive each run's hits in turn. */
size_t tpx_service_device_bytes(const tpx_service* sv);
tpx_status tpx_service_set_segment(tpx_service* sv, uint32_t q);
tpx_status tpx_service_replay(tpx_service* sv, const uint64_t* pk, size_t n, size_t chunk,
                              double pkts_per_s, tpx_hit* hits, size_t hit_cap, float* lat_ms_h,
                              size_t lat_cap, size_t* n_chunks_h, uint64_t* n_runs_h,
                              void* stream);

/* Several independent request streams at once (the streaming workload
 * served to many clients).  A server holds open slots, each an independent
 * tpx_service (its own unwrap state, trigger window, ring and staging); a
 * slot is admitted only while its device memory fits the server's HBM budget,
 * and slot k's runs go to HIP stream k mod n_streams of the server, so runs of
 * different slots issued from different host threads overlap on the GPU.
 * Slots share no state: a slot's hits are the ones it gives alone.
 *   tpx_server_create  hbm_budget_bytes: device memory the slots may hold
 *                       together; n_streams: 1..64 HIP streams.
 *   tpx_server_open    a new slot for a stream with parameters p_h (NULL:
 *                       the server's) whose chunks hold at most
 *                       max_batch_pkts words, ring_pkts of admission ring
 *                       (as tpx_service_create); *slot_h its number (the
 *                       lowest free), *bytes_h (may be NULL) its device
 *                       memory.  TPX_ECAPACITY when that exceeds the free
 *                       budget (nothing stays allocated).
 *   tpx_server_submit / tpx_server_run  tpx_service_submit / _run on the
 *                       slot (run on the slot's HIP stream; synchronises it).
 *   tpx_server_close   frees the slot and returns its memory to the budget.
 * Calls on one slot follow the service's rules; calls on different slots may
 * overlap. */
typedef struct tpx_server tpx_server;
tpx_status tpx_server_create(const tpx_params* p_h, size_t hbm_budget_bytes, int n_streams,
                             tpx_server** out_h);
tpx_status tpx_server_open(tpx_server* sr, const tpx_params* p_h, size_t max_batch_pkts,
                           size_t ring_pkts, uint32_t* slot_h, size_t* bytes_h);
tpx_status tpx_server_submit(tpx_server* sr, uint32_t slot, const uint64_t* chunk, size_t n_pkts,
                             int chunk_on_device, uint64_t* seq_h, void* stream);
tpx_status tpx_server_run(tpx_server* sr, uint32_t slot, int flush, tpx_hit* hits,
                          size_t hit_cap, size_t* n_hits_h, uint64_t* n_done_h,
                          tpx_stats* stats_h);
tpx_status tpx_server_close(tpx_server* sr, uint32_t slot);
size_t tpx_server_free_bytes(tpx_server* sr);
void tpx_server_destroy(tpx_server* sr);

/* Learned centroider / multiplicity splitter.  A small network reads a 7 x 7
 * patch around every hit and predicts up to two hits and their multiplicity;
 * it is trained on clusters with known truth by the gradient and update
 * calls below.  The ToT-weighted centroid (Sec. V, Centroiding, Eq. 9) places
 * the patch and stays the fallback.  All arrays are device memory; every call
 * is ordered on `stream`.
 *
 * Patch of a hit: centred on pixel (floor(x + 1/2), floor(y + 1/2)) of its
 * fp32 centroid; feature c = iy * 7 + ix (ix, iy = pixel - centre + 3 in
 * 0..6) holds min(summed ToT, 1023) / 1024 and feature 49 + c the pixel's
 * earliest ToA minus the hit's toa_first, in 64-tick units (0 for an empty
 * pixel); pixels outside the window are left out.  Features are bfloat16
 * (round to nearest even).
 *   tpx_patches  ev, labels, n_ev: events and their labels (tpx_cluster);
 *                hits, n_hits: their hits in (shot, label) order
 *                (tpx_centroid); feat: bfloat16 [n_hits][98] out;
 *                ws: tpx_patch_workspace_bytes(n_hits) bytes.  TPX_EINVAL
 *                when an event's (shot, label) has no hit.  Synchronises.
 *
 * Network: params is fp32 [93192], packed W1[256][98], b1[256], W2[256][256],
 * b2[256], W3[8][256], b3[8] (W as [out][in]); h1 = relu(W1 f + b1),
 * h2 = relu(W2 h1 + b2), o = W3 h2 + b3, with bfloat16 features, weights and
 * hidden activations on the matrix cores and fp32 accumulation and biases.
 * o[0..2] and o[3..5] are hits A and B as corrections to the hit's weighted
 * centroid (x - hit.x, y - hit.y, (t - toa_first * 1.5625 ns) / 10 ns), o[6]
 * and o[7] the logits of one and two hits: all-zero outputs reproduce the
 * weighted centroid.
 *   tpx_mlp_forward  out: fp32 [n][8]; ws: tpx_mlp_workspace_bytes(min(n,
 *                    65536)) bytes.
 *   tpx_mlp_grad     gradient of the mean loss over a batch of n samples into
 *                    grad (fp32 [93192]): per sample the squared error of hit
 *                    A (one hit) or of the cheaper assignment of A and B to
 *                    the two true hits (two hits), plus the cross entropy of
 *                    the logits.  truth: fp32 [n][2][3] absolute (x, y in
 *                    pixels, t in ns; row 1 ignored for one hit); mult:
 *                    1 or 2 per sample; hits: the samples' hits (patch
 *                    centre, toa_first).  *loss_h (host, may be NULL: then
 *                    no synchronisation) = mean loss.  ws:
 *                    tpx_mlp_workspace_bytes(n) bytes.
 *   tpx_mlp_adam     one Adam step (step counts from 1) on params with
 *                    moments m, v (fp32, zero at the start).
 *   tpx_mlp_refine   refined: fp32 [n][8] = absolute x, y, t_ns of hits A
 *                    and B, then the probability p of two hits, then 0.  When
 *                    p <= 1/2 (a single hit) x, y stay the weighted
 *                    centroid's; t always comes from the network. */
size_t tpx_patch_workspace_bytes(size_t n_hits);
tpx_status tpx_patches(tpx_events ev, const uint32_t* labels, size_t n_ev, const tpx_hit* hits,
                       size_t n_hits, uint16_t* feat, void* ws, size_t ws_bytes, void* stream);
/*   tpx_stream_patches  the same patches for the n_hits hits that the last
 *                       tpx_process_stream call on s wrote (hits: that
 *                       call's output, n_hits its count), taken from the
 *                       stream's own copy of the call's events (valid until
 *                       the next call, set_state or autotune on s): the
 *                       refinement step of the streaming loop.  ws:
 *                       tpx_stream_patch_workspace_bytes(n_hits) bytes.
 *                       TPX_EINVAL without such a call or with another
 *                       count.  Synchronises. */
size_t tpx_stream_patch_workspace_bytes(size_t n_hits);
/*   tpx_stream_set_patches  enable (1) or disable (0) recording, during each
 *                       tpx_process_stream call on s, the hit of every event
 *                       (4 bytes per event) that tpx_stream_patches needs
 *                       after the fused kernel; enable it before the call
 *                       whose hits are to be patched. */
tpx_status tpx_stream_set_patches(tpx_stream* s, int enable);
tpx_status tpx_stream_patches(tpx_stream* s, const tpx_hit* hits, size_t n_hits, uint16_t* feat,
                              void* ws, size_t ws_bytes, void* stream);
size_t tpx_mlp_workspace_bytes(size_t batch);
tpx_status tpx_mlp_forward(const float* params, const uint16_t* feat, size_t n, float* out,
                           void* ws, size_t ws_bytes, void* stream);
tpx_status tpx_mlp_grad(const float* params, const uint16_t* feat, const tpx_hit* hits,
                        const float* truth, const uint8_t* mult, size_t n, float* grad,
                        float* loss_h, void* ws, size_t ws_bytes, void* stream);
tpx_status tpx_mlp_adam(float* params, float* m, float* v, const float* grad, size_t n_param,
                        uint64_t step, float lr, float beta1, float beta2, float eps,
                        void* stream);
tpx_status tpx_mlp_refine(const tpx_hit* hits, const float* out, size_t n, float* refined,
                          void* stream);

const char* tpx_status_str(tpx_status st);
const char* tpx_last_error(void); /* thread-local detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* TPX_H */
