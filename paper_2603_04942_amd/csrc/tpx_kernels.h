// Kernel argument blocks and launch wrappers of libtpx (internal).
#pragma once

#include "tpx_internal.h"

namespace tpx {

struct AssignArgs {
    const uint64_t* pk;
    uint64_t n;
    uint32_t sub;
    uint32_t tof_max;
    uint64_t jump;
    const TileEntry* entries;
    const TileAcc* sums;       // per-tile summaries (trigger count of each tile)
    const uint64_t* tab;       // trigger table: [window triggers..., new triggers...]
    uint64_t n_win;            // window triggers in front of this call's
    const unsigned long long* n_trig_dev;  // triggers decoded by this call
    uint64_t first_open;       // table index of the first shot still open
    uint64_t tab_has_before;   // triggers existed before tab[0]
    // packed output (stream path)
    uint64_t* ev;
    uint64_t ev_off;           // events already in front of this chunk's (carry)
    uint64_t ev_cap;
    uint32_t* shot_out;        // optional: table index of every kept event
    uint32_t* shot_cnt;        // kept events per table index (stream path)
    // structure-of-arrays output (tpx_decode)
    tpx_events soa;
    uint64_t shot_base;        // global index of tab[0]
    uint64_t carry_last1;      // table index + 1 of the last event in front (0 = none)
    uint64_t* lb_status;       // zeroed, one word per tile
    DevResults* res;
    // staged packed output (launch_assign_staged): tile t writes its kept
    // events at ev[t * kTilePkts ..] and its count, smallest and largest
    // kept shot (+1) and statistics here
    uint32_t *tile_cnt, *tile_lo, *tile_hi;
    unsigned long long* tile_stat;  // 8 per tile
};

struct ClusterArgs {
    const uint64_t* ev;        // packed events in group order (stream path)
    tpx_events soa;            // original events (event mode)
    const uint32_t* perm;      // group-order position -> original position, or null
    const uint32_t* grp_off;   // first position of each group, [n_grp + 1]
    const uint32_t* seg_lo;    // first group of each segment, [n_seg + 1] (k_seg_table)
    const uint32_t* grp_shot;  // group -> table index (stream) or shot value; null = identity
    const unsigned long long* n_ev_dev;
    const unsigned long long* n_grp_dev;
    uint32_t q;                // segment stride in events
    uint32_t dxy, dt;
    const uint64_t* carry_gidx;
    uint64_t n_carry, ev_base;
    const uint64_t* tab;
    uint64_t tab_base;
    const float* walk;
    tpx_hit* hits;
    uint64_t hit_cap;
    uint32_t* labels;          // event mode: label of every event
    uint32_t* rank;            // stream mode: component rank of every event in its segment
    uint32_t* seg_cnt;         // stream mode: components per segment
    const uint32_t* seg_off;   // stream mode: exclusive prefix of seg_cnt, [n_seg + 1]
    DevResults* res;
    const unsigned long long* skip;  // non-zero: do nothing (events not in shot order)
    // per-event scratch for segments that do not fit in LDS
    uint32_t *g_parent, *g_chain, *g_next, *g_t, *g_sl, *g_xy;
    uint64_t* g_acc;           // 8 words per event
    // fused stream kernel (launch_cluster_fused)
    tpx_hit* hits_tmp;         // staging: hit r of a segment at its first event + r
    uint32_t* hit_index;       // optional: hit of every event (call-relative), or null
    uint32_t* defer_list;      // routed variant: segments left to the persistent launch
};

void launch_tile_summary(const uint64_t* pk, uint64_t n, uint32_t sub, uint64_t jump,
                         TileAcc* sums, uint64_t* tdc_slot, hipStream_t s);
// blk holds 2 * ceil(ntiles / 1024) entries
void launch_tile_scan(const TileAcc* sums, uint64_t ntiles, TileAcc init, int64_t pe0, int64_t te0,
                      uint64_t jump, TileAcc* partial, TileAcc* blk, DevResults* res, hipStream_t s);
void launch_trig_unwrap(const TileAcc* sums, const TileAcc* partial, const TileAcc* blk,
                        const uint64_t* slot, uint64_t ntiles, int64_t pe0, int64_t te0,
                        uint64_t jump, TileEntry* entries, uint64_t* tab, DevResults* res,
                        hipStream_t s);
uint64_t tile_scan_blocks(uint64_t ntiles);
void launch_assign(const AssignArgs& a, bool soa, hipStream_t s);
// Stream path without a look-back over tiles: every tile writes its kept
// events (and shots, when a.shot_out) to its own range of a.ev / a.shot_out
// (staging) with per-tile counts; then launch_assign_place moves them to
// ev_out[ev_off + prefix] (shot_out_final likewise), checks the shot order
// across tiles and reduces the statistics.  tile_off: ntiles + 1 words
// (exclusive prefix of tile_cnt, filled by the caller's scan).
void launch_assign_staged(const AssignArgs& a, hipStream_t s);
void launch_assign_place(const AssignArgs& a, const uint32_t* tile_off, uint64_t* ev_out,
                         uint64_t ev_off, uint64_t ev_cap, uint32_t* shot_out_final,
                         hipStream_t s);
void launch_cluster(const ClusterArgs& a, bool event_mode, uint64_t grid, hipStream_t s);
// segment table of a group offset array (see ClusterArgs::seg_lo); needs
// max_events / q + 2 entries
void launch_seg_table(const uint32_t* grp_off, const unsigned long long* n_grp_dev,
                      const unsigned long long* n_ev_dev, const unsigned long long* skip,
                      uint32_t q, uint64_t max_groups, uint32_t* seg_lo, DevResults* res,
                      hipStream_t s);
// stream mode: moments and hits of the components found by launch_cluster
void launch_seg_centroid(const ClusterArgs& a, uint64_t grid, hipStream_t s);
// stream mode, radius 1, times of flight below 2^16: components, moments and
// hits of every segment in one launch, hits staged at each segment's own
// range of a.hits_tmp and its component count in seg_cnt; `variant` selects
// the image height, workgroup size and LDS capacity (fused_variants()); the
// routed variant clusters segments beyond 2,048 events in a second,
// persistent launch of list_grid workgroups over the segments the first one
// appended to defer_list (one entry per segment: grid words; the counters
// res->aux_ticket and res->seg_ticket must be zero).
// Then a prefix sum of seg_cnt into seg_off, and launch_hit_compact moves the
// hits to their final place (and sets res->n_hits).
void launch_cluster_fused(const ClusterArgs& a, uint64_t grid, int variant, uint32_t* defer_list,
                          uint32_t list_grid, hipStream_t s);
void launch_hit_compact(const ClusterArgs& a, uint64_t grid, hipStream_t s);

// The fast stream path of one chunk in one persistent launch (tpx_cluster.hip,
// k_stream_chunk): `a` and `c` as for the separate launches (a staged, with
// the staging buffers; c with the group table, segment table and the counts
// of the call's results), plus what the prefix, close rule and carry need.
// qs: kQWords counters, zero before the first launch (each launch leaves them
// zero).  At most chunk_max_tiles() tiles.
struct ChunkArgs {
    AssignArgs a;
    ClusterArgs c;
    TileAcc* sums;
    uint64_t* tdc_slot;
    TileEntry* entries;
    uint64_t* tab_new;                 // this call's triggers: tab + n_win
    TileAcc init;                      // counter state in force at the call's start
    int64_t pe0, te0;
    uint32_t* tile_off;                // ntiles + 1
    uint64_t* ev;                      // kept events: carried, then this call's
    uint64_t ev_cap;
    const uint64_t* c_ev_in;
    const uint32_t* c_shot_in;
    uint64_t n_carry;
    uint32_t carry_rebase;
    int flush;
    uint64_t max_t_plus1_prev, slack;
    const uint64_t* c_gidx_in;
    uint64_t* c_ev_out;
    uint32_t* c_shot_out;
    uint64_t* c_gidx_out;
    uint64_t carry_cap;
    unsigned int* qs;
    uint32_t ntiles, seg_grid;
};
// p_dev: a device copy of p, complete when the launch runs (stream order)
void launch_stream_chunk(const ChunkArgs& p, const ChunkArgs* p_dev, uint32_t grid, hipStream_t s);
uint32_t chunk_max_tiles();
uint32_t chunk_queue_words();
int fused_variants();
const char* fused_variant_name(int variant);
// patches of the hits written by the stream call whose cluster arguments are
// `a` (tpx_learn.hip); acc: u32 [n_hits * 98 + n_hits] scratch, err: 1 word
// (fused: the call recorded the hit of every event in a.hit_index)
void launch_stream_patches(const ClusterArgs& a, uint64_t grid, bool fused, const tpx_hit* hits,
                           uint64_t n_hits, uint32_t* acc, uint16_t* feat, int* err,
                           hipStream_t s);
// event mode, the paper's local-maximum hits: count pass (write = false,
// fills seg_cnt), then write pass (hits at seg_off[k] + rank)
void launch_paper(const ClusterArgs& a, const uint64_t* trig, bool write, uint64_t grid,
                  hipStream_t s);
// workgroups needed to cover every segment of up to max_events events
uint64_t cluster_grid(uint64_t max_events, uint32_t q);
int cluster_capacity();

// sets the text returned by tpx_last_error and returns st (tpx_api.hip)
tpx_status report(tpx_status st, const char* msg);

// utilities (tpx_util.hip)
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void launch_fill_u32_dev(uint32_t* p, uint32_t v, uint64_t base, const unsigned long long* n_dev,
                         uint64_t extra, hipStream_t s);
void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s);
// out[0..n] = exclusive prefix of in[0..n), out[n] = total; n = *n_dev if n_dev
void launch_scan_u32(const uint32_t* in, uint32_t* out, uint64_t n_host,
                     const unsigned long long* n_dev, uint32_t* block_tmp, hipStream_t s);
void launch_close(const uint64_t* tab, const unsigned long long* n_trig_dev, uint64_t n_win,
                  uint64_t first_open, int flush, uint64_t max_t_plus1_prev, uint64_t tof_max,
                  uint64_t slack, const uint32_t* shot_off, DevResults* res, hipStream_t s);
void launch_set_rows(DevResults* res, uint64_t n_win, hipStream_t s);
void launch_check_events(tpx_events ev, uint64_t n, DevResults* res, hipStream_t s);
// groups of equal keys in a sorted key array: grp_off[G+1], grp_shot[G], res->n_groups = G
void launch_boundaries(const uint32_t* sorted_key, uint64_t n, uint32_t* flags, uint32_t* scan,
                       uint32_t* block_tmp, uint32_t* grp_off, uint32_t* grp_shot,
                       DevResults* res, hipStream_t s);
// fallback stream path: closed groups / events from sorted keys and the close index
void launch_close_sorted(const uint32_t* sorted_key, uint64_t n, const uint32_t* grp_shot,
                         DevResults* res, hipStream_t s);
void radix_sort_pairs(uint32_t* key, uint32_t* val, uint32_t* key2, uint32_t* val2,
                      uint32_t* flags, uint32_t* scan, uint32_t* block_tmp, uint64_t n, int bits,
                      hipStream_t s, uint32_t** key_out, uint32_t** val_out);
void launch_iota_u32(uint32_t* p, uint64_t n, hipStream_t s);
void launch_gather_keys(const uint32_t* shot, const uint32_t* perm, uint32_t* out, uint64_t n,
                        hipStream_t s);
void launch_gather_packed(const uint64_t* ev, const uint32_t* perm, uint64_t* out, uint64_t n,
                          hipStream_t s);
void launch_carry_in(const uint64_t* c_ev, const uint32_t* c_shot, uint64_t n_carry,
                     uint32_t rebase, uint64_t* ev, uint32_t* shot_arr, uint32_t* shot_cnt,
                     hipStream_t s);
void launch_carry_out(const uint64_t* ev, const uint32_t* perm, const uint32_t* shot_arr,
                      const uint32_t* shot_off, const unsigned long long* n_rows_dev,
                      const unsigned long long* n_close_ev, const unsigned long long* n_kept,
                      const uint64_t* carry_gidx_in, uint64_t n_carry, uint64_t ev_base,
                      uint64_t* c_ev, uint32_t* c_shot, uint64_t* c_gidx, uint64_t carry_cap,
                      DevResults* res, hipStream_t s);
void launch_copy_u64(const uint64_t* src, uint64_t* dst, uint64_t n, hipStream_t s);
// centroids of given labels (tpx_centroid)
void launch_cent_init(uint64_t* acc, uint64_t n, hipStream_t s);
void launch_cent_accum(tpx_events ev, const uint32_t* labels, uint64_t n, const uint64_t* trig,
                       uint64_t n_trig, const float* walk, uint64_t* acc, DevResults* res,
                       hipStream_t s);
void launch_root_flags(const uint32_t* labels, uint64_t n, uint32_t* flags, hipStream_t s);
void launch_compact_roots(const uint32_t* flags, const uint32_t* scan, uint64_t n,
                          uint32_t* roots, hipStream_t s);
void launch_cent_emit(tpx_events ev, const uint32_t* order, uint64_t n_roots,
                      const uint64_t* acc, const uint64_t* trig, const float* walk,
                      tpx_hit* hits, uint64_t hit_cap, hipStream_t s);

}  // namespace tpx
