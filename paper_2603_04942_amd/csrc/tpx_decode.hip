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
#include "tpx_decode_dev.h"

namespace tpx {
__global__ __launch_bounds__(kSumThreads) void k_tile_summary(const uint64_t* __restrict__ pk,
                                                             uint64_t n, uint32_t sub,
                                                             uint64_t jump, TileAcc* sums,
                                                             uint64_t* tdc_slot) {
    __shared__ RunSum wbuf[kSumWaves];
    __shared__ uint32_t tmp[kSumWaves + 1];
    tile_summary_body(pk, n, sub, jump, sums, tdc_slot, blockIdx.x, wbuf, tmp);
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

// One thread per tile.
__global__ void k_trig_unwrap(const TileAcc* __restrict__ sums, const TileAcc* __restrict__ partial,
                              const TileAcc* __restrict__ blk, const uint64_t* __restrict__ tdc_slot,
                              uint64_t ntiles, uint64_t nblk, int64_t pe0, int64_t te0,
                              uint64_t jump, TileEntry* entries, uint64_t* tab, DevResults* res) {
    const uint64_t tile = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    const TileAcc pre = acc_combine(blk[nblk + tile / kScanTiles], partial[tile], jump);
    // blk[nblk] is the state in force at the front of block 0: the initial state
    unwrap_tile(pre, blk[nblk].ntrig, tile, sums, tdc_slot, pe0, te0, jump, entries, tab, res);
}

template <bool kSoA, bool kStaged = false>
__global__ __launch_bounds__(kTileThreads) void k_assign(AssignArgs a) {
    __shared__ AssignLds<kTileThreads, kSoA> L;
    assign_body<kSoA, kStaged, kTileThreads>(a, blockIdx.x, L);
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

__global__ __launch_bounds__(kPlaceThreads) void k_assign_place(AssignArgs a, const uint32_t* tile_off,
                                                                uint64_t* ev_out, uint64_t ev_off,
                                                                uint64_t ev_cap,
                                                                uint32_t* shot_final,
                                                                uint64_t ntiles) {
    place_tile(a, tile_off, ev_out, ev_off, ev_cap, shot_final, ntiles, blockIdx.x, kPlaceThreads);
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
