// Small device utilities of libtpx: fills, prefix sums, the close rule,
// the stable split sort used when events are not in shot order, carry
// copies between stream chunks, and centroids of externally given labels.
#include "tpx_util_dev.h"

namespace tpx {

constexpr int kScanBlocks = 256;
constexpr int kScanThreads = 1024;

static inline unsigned grid_for(uint64_t n, int threads, unsigned cap = 65535u * 4) {
    uint64_t g = (n + threads - 1) / threads;
    if (g == 0) g = 1;
    return (unsigned)(g > cap ? cap : g);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
// p[0 .. base + *n_dev + extra) = v, the count read on the device
__global__ void k_fill_u32_dev(uint32_t* p, uint32_t v, uint64_t base,
                               const unsigned long long* n_dev, uint64_t extra) {
    const uint64_t n = base + *n_dev + extra;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
void launch_fill_u32_dev(uint32_t* p, uint32_t v, uint64_t base, const unsigned long long* n_dev,
                         uint64_t extra, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32_dev, dim3(256), dim3(256), 0, s, p, v, base, n_dev, extra);
}

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
}
void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
}

__global__ void k_copy_u64(const uint64_t* src, uint64_t* dst, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
void launch_copy_u64(const uint64_t* src, uint64_t* dst, uint64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_copy_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, src, dst, n);
}

__global__ void k_iota_u32(uint32_t* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}
void launch_iota_u32(uint32_t* p, uint64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_iota_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n);
}

// ------------------------------------------------------------ prefix sums
// Reduce-then-scan over kScanBlocks contiguous chunks; n may live on the device.
__device__ inline uint64_t scan_n(uint64_t n_host, const unsigned long long* n_dev) {
    return n_dev ? (uint64_t)*n_dev : n_host;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* in, uint64_t n_host,
                                                             const unsigned long long* n_dev,
                                                             uint32_t* block_tmp) {
    const uint64_t n = scan_n(n_host, n_dev);
    const uint64_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
    const uint64_t lo = min<uint64_t>(n, (uint64_t)blockIdx.x * chunk);
    const uint64_t hi = min<uint64_t>(n, lo + chunk);
    uint32_t s = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kScanThreads) s += in[i];
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    __shared__ uint32_t w[kScanThreads / 64];
    if (__lane_id() == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kScanThreads / 64; ++k) t += w[k];
        block_tmp[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kScanBlocks) void k_scan_blocks(uint32_t* block_tmp) {
    __shared__ uint32_t tmp[kScanBlocks / 64 + 1];
    uint32_t tot;
    const uint32_t v = block_tmp[threadIdx.x];
    const uint32_t p = wg_count_scan<kScanBlocks>(v, tmp, &tot);
    block_tmp[kScanBlocks + threadIdx.x] = p;
    if (threadIdx.x == 0) block_tmp[2 * kScanBlocks] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* in, uint32_t* out,
                                                           uint64_t n_host,
                                                           const unsigned long long* n_dev,
                                                           const uint32_t* block_tmp) {
    __shared__ uint32_t tmp[kScanThreads / 64 + 1];
    const uint64_t n = scan_n(n_host, n_dev);
    const uint64_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
    const uint64_t lo = min<uint64_t>(n, (uint64_t)blockIdx.x * chunk);
    const uint64_t hi = min<uint64_t>(n, lo + chunk);
    uint32_t run = block_tmp[kScanBlocks + blockIdx.x];
    for (uint64_t base = lo; base < hi; base += kScanThreads) {
        const uint64_t i = base + threadIdx.x;
        const uint32_t v = i < hi ? in[i] : 0u;
        uint32_t tot;
        const uint32_t p = wg_count_scan<kScanThreads>(v, tmp, &tot);
        if (i < hi) out[i] = run + p;
        run += tot;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = block_tmp[2 * kScanBlocks];
}

void launch_scan_u32(const uint32_t* in, uint32_t* out, uint64_t n_host,
                     const unsigned long long* n_dev, uint32_t* block_tmp, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_reduce, dim3(kScanBlocks), dim3(kScanThreads), 0, s, in, n_host, n_dev,
                       block_tmp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlocks), 0, s, block_tmp);
    hipLaunchKernelGGL(k_scan_down, dim3(kScanBlocks), dim3(kScanThreads), 0, s, in, out, n_host,
                       n_dev, block_tmp);
}

// the close rule of close_rule (tpx_util_dev.h)
__global__ void k_close(const uint64_t* tab, const unsigned long long* n_trig_dev, uint64_t n_win,
                        uint64_t first_open, int flush, uint64_t max_t_plus1_prev,
                        uint64_t tof_max, uint64_t slack, const uint32_t* shot_off,
                        DevResults* res) {
    close_rule(tab, n_trig_dev, n_win, first_open, flush, max_t_plus1_prev, tof_max, slack,
               shot_off, res);
}
void launch_close(const uint64_t* tab, const unsigned long long* n_trig_dev, uint64_t n_win,
                  uint64_t first_open, int flush, uint64_t max_t_plus1_prev, uint64_t tof_max,
                  uint64_t slack, const uint32_t* shot_off, DevResults* res, hipStream_t s) {
    hipLaunchKernelGGL(k_close, dim3(1), dim3(1), 0, s, tab, n_trig_dev, n_win, first_open, flush,
                       max_t_plus1_prev, tof_max, slack, shot_off, res);
}

__global__ void k_set_rows(DevResults* res, uint64_t n_win) { res->n_groups = n_win + res->n_trig; }
void launch_set_rows(DevResults* res, uint64_t n_win, hipStream_t s) {
    hipLaunchKernelGGL(k_set_rows, dim3(1), dim3(1), 0, s, res, n_win);
}

// Fallback path: events sorted by table index; closed events and groups are
// those with index below n_close_grp (as computed by k_close).
__global__ void k_close_sorted(const uint32_t* key, uint64_t n, const uint32_t* grp_shot,
                               DevResults* res) {
    const uint64_t s_close = res->n_close_grp;
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t m = (lo + hi) >> 1;
        if (key[m] < s_close) lo = m + 1; else hi = m;
    }
    res->n_close_ev = lo;
    const uint64_t G = res->n_groups;
    uint64_t a = 0, b = G;
    while (a < b) {
        const uint64_t m = (a + b) >> 1;
        if (grp_shot[m] < s_close) a = m + 1; else b = m;
    }
    res->n_close_list = a;
}
void launch_close_sorted(const uint32_t* sorted_key, uint64_t n, const uint32_t* grp_shot,
                         DevResults* res, hipStream_t s) {
    hipLaunchKernelGGL(k_close_sorted, dim3(1), dim3(1), 0, s, sorted_key, n, grp_shot, res);
}

// Event-mode input check: value ranges, shot order and the largest shot.
__global__ void k_check_events(tpx_events ev, uint64_t n, DevResults* res) {
    bool bad = false, uns = false;
    uint32_t mk = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (ev.x[i] > 255 || ev.y[i] > 255 || ev.tot[i] > 1023) bad = true;
        const uint32_t s = ev.shot[i];
        if (i > 0 && s < ev.shot[i - 1]) uns = true;
        mk = max(mk, s);
    }
    if (bad) atomicOr(&res->err, (unsigned long long)kErrInput);
    if (uns) atomicOr(&res->unsorted, 1ull);
    for (int d = 32; d > 0; d >>= 1) mk = max(mk, (uint32_t)__shfl_xor(mk, d, 64));
    if (__lane_id() == 0) atomicMax(&res->max_key, (unsigned long long)mk);
}
void launch_check_events(tpx_events ev, uint64_t n, DevResults* res, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_check_events, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, ev, n, res);
}

// ------------------------------------------------------------ groups
__global__ void k_bound_flags(const uint32_t* key, uint64_t n, uint32_t* flags) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        flags[i] = (i == 0 || key[i] != key[i - 1]) ? 1u : 0u;
}
__global__ void k_bound_scatter(const uint32_t* key, uint64_t n, const uint32_t* flags,
                                const uint32_t* scan, uint32_t* grp_off, uint32_t* grp_shot,
                                DevResults* res) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (flags[i]) {
            grp_off[scan[i]] = (uint32_t)i;
            grp_shot[scan[i]] = key[i];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t G = n ? scan[n] : 0u;
        grp_off[G] = (uint32_t)n;
        res->n_groups = G;
    }
}
void launch_boundaries(const uint32_t* sorted_key, uint64_t n, uint32_t* flags, uint32_t* scan,
                       uint32_t* block_tmp, uint32_t* grp_off, uint32_t* grp_shot,
                       DevResults* res, hipStream_t s) {
    if (n) {
        hipLaunchKernelGGL(k_bound_flags, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, sorted_key,
                           n, flags);
        launch_scan_u32(flags, scan, n, nullptr, block_tmp, s);
    }
    hipLaunchKernelGGL(k_bound_scatter, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, sorted_key,
                       n, flags, scan, grp_off, grp_shot, res);
}

// ------------------------------------------------------------ stable sort
// One binary digit per pass: zeros keep their order in front, ones behind.
__global__ void k_split_flags(const uint32_t* key, uint64_t n, int bit, uint32_t* flags) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        flags[i] = ((key[i] >> bit) & 1u) ? 0u : 1u;
}
__global__ void k_split_scatter(const uint32_t* key, const uint32_t* val, uint64_t n,
                                const uint32_t* flags, const uint32_t* scan, uint32_t* key2,
                                uint32_t* val2) {
    const uint64_t zeros = scan[n];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t d = flags[i] ? scan[i] : zeros + i - scan[i];
        key2[d] = key[i];
        val2[d] = val[i];
    }
}
// 4-bit digits: blocks of 4,096 pairs (256 threads x 16 consecutive pairs).
// Pass = count (digit totals of every block, digit-major: cnt[d * nb + b]),
// exclusive prefix of the counts (every (digit, block) start), scatter: in a
// block, the exclusive prefix of the per-thread digit counts in digit-major
// order gives each thread the rank of its first pair of each digit among
// the block's pairs of that digit; the thread then writes its pairs in order
// (stable).
constexpr int kRsThreads = 256, kRsItems = 16, kRsTile = kRsThreads * kRsItems;
constexpr int kRsBits = 4, kRsDigits = 1 << kRsBits;

__global__ __launch_bounds__(kRsThreads) void k_rs_count(const uint32_t* key, uint64_t n, int sh,
                                                         uint32_t mask, uint32_t* cnt,
                                                         uint64_t nb) {
    __shared__ uint32_t h[kRsDigits];
    if (threadIdx.x < kRsDigits) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t b = blockIdx.x, i0 = b * kRsTile + (uint64_t)threadIdx.x * kRsItems;
    for (int j = 0; j < kRsItems; ++j)
        if (i0 + j < n) atomicAdd(&h[(key[i0 + j] >> sh) & mask], 1u);
    __syncthreads();
    if (threadIdx.x < kRsDigits) cnt[(uint64_t)threadIdx.x * nb + b] = h[threadIdx.x];
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint32_t* key, const uint32_t* val,
                                                           uint64_t n, int sh, uint32_t mask,
                                                           const uint32_t* off, uint64_t nb,
                                                           uint32_t* key2, uint32_t* val2) {
    __shared__ uint32_t c[kRsDigits * kRsThreads];  // [digit][thread], then cursors
    __shared__ uint32_t dstart[kRsDigits];           // the block's first position of each digit
    __shared__ uint32_t tmp[kRsThreads / 64 + 1];
    const uint32_t t = threadIdx.x;
    const uint64_t b = blockIdx.x, i0 = b * kRsTile + (uint64_t)t * kRsItems;
    for (int d = 0; d < kRsDigits; ++d) c[d * kRsThreads + t] = 0;
    for (int j = 0; j < kRsItems; ++j)
        if (i0 + j < n) ++c[((key[i0 + j] >> sh) & mask) * kRsThreads + t];
    __syncthreads();
    // exclusive prefix over the 4,096 counts in digit-major order: thread t
    // takes entries [16 t, 16 t + 16)
    uint32_t v[kRsItems], sum = 0;
    for (int k = 0; k < kRsItems; ++k) {
        v[k] = sum;
        sum += c[t * kRsItems + k];
    }
    uint32_t total;
    const uint32_t base = wg_count_scan<kRsThreads>(sum, tmp, &total);
    __syncthreads();
    for (int k = 0; k < kRsItems; ++k) c[t * kRsItems + k] = base + v[k];
    __syncthreads();
    if (t < kRsDigits) dstart[t] = c[t * kRsThreads];
    __syncthreads();
    // c[d][t] = pairs of the block before thread t's first pair of digit d
    // (all smaller digits, then digit d in earlier threads); minus the
    // block's start of digit d it is the rank within digit d; thread t then
    // advances its own cursor c[d][t]
    for (int j = 0; j < kRsItems; ++j) {
        const uint64_t i = i0 + j;
        if (i >= n) break;
        const uint32_t k = key[i], d = (k >> sh) & mask;
        const uint32_t r = c[d * kRsThreads + t] - dstart[d];
        ++c[d * kRsThreads + t];
        const uint64_t dst = (uint64_t)off[(uint64_t)d * nb + b] + r;
        key2[dst] = k;
        val2[dst] = val[i];
    }
}

void radix_sort_pairs(uint32_t* key, uint32_t* val, uint32_t* key2, uint32_t* val2,
                      uint32_t* flags, uint32_t* scan, uint32_t* block_tmp, uint64_t n, int bits,
                      hipStream_t s, uint32_t** key_out, uint32_t** val_out) {
    // 4-bit passes while the digit counts fit the buffers (flags: n + 1
    // words, scan: n + 2), else (fewer than 32 pairs) one bit at a time
    const uint64_t nb = (n + kRsTile - 1) / kRsTile;
    const bool wide = n >= 32 && (uint64_t)kRsDigits * nb + 1 <= n + 1;
    for (int b = 0; wide && b < bits; b += kRsBits) {
        const int w = bits - b < kRsBits ? bits - b : kRsBits;
        const uint32_t mask = (1u << w) - 1u;
        hipLaunchKernelGGL(k_rs_count, dim3((unsigned)nb), dim3(kRsThreads), 0, s, key, n, b, mask,
                           flags, nb);
        launch_scan_u32(flags, scan, (uint64_t)kRsDigits * nb, nullptr, block_tmp, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(kRsThreads), 0, s, key, val, n, b,
                           mask, scan, nb, key2, val2);
        uint32_t* t = key;
        key = key2;
        key2 = t;
        t = val;
        val = val2;
        val2 = t;
    }
    for (int b = 0; !wide && b < bits && n > 1; ++b) {
        hipLaunchKernelGGL(k_split_flags, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, key, n, b,
                           flags);
        launch_scan_u32(flags, scan, n, nullptr, block_tmp, s);
        hipLaunchKernelGGL(k_split_scatter, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, key, val,
                           n, flags, scan, key2, val2);
        uint32_t* t = key;
        key = key2;
        key2 = t;
        t = val;
        val = val2;
        val2 = t;
    }
    *key_out = key;
    *val_out = val;
}

__global__ void k_gather_keys(const uint32_t* shot, const uint32_t* perm, uint32_t* out, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = shot[perm[i]];
}
void launch_gather_keys(const uint32_t* shot, const uint32_t* perm, uint32_t* out, uint64_t n,
                        hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_gather_keys, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, shot, perm, out, n);
}
__global__ void k_gather_packed(const uint64_t* ev, const uint32_t* perm, uint64_t* out, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = ev[perm[i]];
}
void launch_gather_packed(const uint64_t* ev, const uint32_t* perm, uint64_t* out, uint64_t n,
                          hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_gather_packed, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ev, perm, out, n);
}

// ------------------------------------------------------------ stream carry
__global__ void k_carry_in(const uint64_t* c_ev, const uint32_t* c_shot, uint64_t n_carry,
                           uint32_t rebase, uint64_t* ev, uint32_t* shot_arr, uint32_t* shot_cnt) {
    carry_in_range(c_ev, c_shot, n_carry, rebase, ev, shot_arr, shot_cnt,
                   (uint64_t)blockIdx.x * blockDim.x + threadIdx.x,
                   (uint64_t)gridDim.x * blockDim.x);
}
void launch_carry_in(const uint64_t* c_ev, const uint32_t* c_shot, uint64_t n_carry,
                     uint32_t rebase, uint64_t* ev, uint32_t* shot_arr, uint32_t* shot_cnt,
                     hipStream_t s) {
    if (n_carry)
        hipLaunchKernelGGL(k_carry_in, dim3(grid_for(n_carry, 256, 1024)), dim3(256), 0, s, c_ev,
                           c_shot, n_carry, rebase, ev, shot_arr, shot_cnt);
}

__global__ void k_carry_out(const uint64_t* ev, const uint32_t* perm, const uint32_t* shot_arr,
                            const uint32_t* shot_off, const unsigned long long* n_rows_dev,
                            const unsigned long long* n_close_ev, const unsigned long long* n_kept,
                            const uint64_t* carry_gidx_in, uint64_t n_carry, uint64_t ev_base,
                            uint64_t* c_ev, uint32_t* c_shot, uint64_t* c_gidx, uint64_t carry_cap,
                            DevResults* res) {
    carry_out_range(ev, perm, shot_arr, shot_off, n_rows_dev, n_close_ev, n_kept, carry_gidx_in,
                    n_carry, ev_base, c_ev, c_shot, c_gidx, carry_cap, res,
                    (uint64_t)blockIdx.x * blockDim.x + threadIdx.x,
                    (uint64_t)gridDim.x * blockDim.x);
}
void launch_carry_out(const uint64_t* ev, const uint32_t* perm, const uint32_t* shot_arr,
                      const uint32_t* shot_off, const unsigned long long* n_rows_dev,
                      const unsigned long long* n_close_ev, const unsigned long long* n_kept,
                      const uint64_t* carry_gidx_in, uint64_t n_carry, uint64_t ev_base,
                      uint64_t* c_ev, uint32_t* c_shot, uint64_t* c_gidx, uint64_t carry_cap,
                      DevResults* res, hipStream_t s) {
    hipLaunchKernelGGL(k_carry_out, dim3(1024), dim3(256), 0, s, ev, perm, shot_arr, shot_off,
                       n_rows_dev, n_close_ev, n_kept, carry_gidx_in, n_carry, ev_base, c_ev,
                       c_shot, c_gidx, carry_cap, res);
}

// ------------------------------------------------- centroids of given labels
constexpr int kAcc = 10;  // W, count, Sx, Sy, St, min ToA, Ux, Uy, Ut, spare

__global__ void k_cent_init(uint64_t* acc, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < kAcc; ++k) acc[kAcc * i + k] = (k == 5) ? ~0ull : 0ull;
    }
}
void launch_cent_init(uint64_t* acc, uint64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_cent_init, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, acc, n);
}

__device__ inline int64_t tof_term(const float* walk, uint32_t tot, int64_t tof) {
    if (walk) return tof * 102400 - llrint((double)walk[tot & 1023u] * 65536.0);
    return tof;
}

__global__ void k_cent_accum(tpx_events ev, const uint32_t* labels, uint64_t n,
                             const uint64_t* trig, uint64_t n_trig, const float* walk,
                             uint64_t* acc, DevResults* res) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t r = labels[i];
        const uint32_t s = ev.shot[i];
        if (r >= n || labels[r] != r || ev.shot[r] != s || s >= n_trig || ev.x[i] > 255 ||
            ev.y[i] > 255 || ev.tot[i] > 1023) {
            atomicOr(&res->err, (unsigned long long)kErrInput);
            continue;
        }
        const uint64_t toa = ev.toa[i];
        const int64_t tof = (int64_t)(toa - trig[s]);
        const uint32_t tot = ev.tot[i], x = ev.x[i], y = ev.y[i];
        unsigned long long* q = (unsigned long long*)acc + kAcc * (uint64_t)r;
        atomicAdd(q + 0, (unsigned long long)tot);
        atomicAdd(q + 1, 1ull);
        atomicAdd(q + 2, (unsigned long long)(tot * x));
        atomicAdd(q + 3, (unsigned long long)(tot * y));
        atomicAdd(q + 4, (unsigned long long)((int64_t)tot * tof_term(walk, tot, tof)));
        atomicMin(q + 5, (unsigned long long)toa);
        atomicAdd(q + 6, (unsigned long long)x);
        atomicAdd(q + 7, (unsigned long long)y);
        atomicAdd(q + 8, (unsigned long long)tof_term(walk, tot, tof));
    }
}
void launch_cent_accum(tpx_events ev, const uint32_t* labels, uint64_t n, const uint64_t* trig,
                       uint64_t n_trig, const float* walk, uint64_t* acc, DevResults* res,
                       hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_cent_accum, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ev, labels,
                              n, trig, n_trig, walk, acc, res);
}

__global__ void k_root_flags(const uint32_t* labels, uint64_t n, uint32_t* flags) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        flags[i] = labels[i] == (uint32_t)i ? 1u : 0u;
}
void launch_root_flags(const uint32_t* labels, uint64_t n, uint32_t* flags, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_root_flags, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, labels, n, flags);
}
__global__ void k_compact_roots(const uint32_t* flags, const uint32_t* scan, uint64_t n,
                                uint32_t* roots) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        if (flags[i]) roots[scan[i]] = (uint32_t)i;
}
void launch_compact_roots(const uint32_t* flags, const uint32_t* scan, uint64_t n,
                          uint32_t* roots, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_compact_roots, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, flags, scan,
                              n, roots);
}

__global__ void k_cent_emit(tpx_events ev, const uint32_t* order, uint64_t n_roots,
                            const uint64_t* acc, const uint64_t* trig, const float* walk,
                            tpx_hit* hits, uint64_t hit_cap) {
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_roots && k < hit_cap;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = order[k];
        const uint64_t* q = acc + kAcc * (uint64_t)i;
        const uint64_t W = q[0], cnt = q[1];
        tpx_hit h;
        const double den = W ? (double)W : (double)cnt;
        const uint64_t sx = W ? q[2] : q[6], sy = W ? q[3] : q[7];
        const int64_t st = (int64_t)(W ? q[4] : q[8]);
        h.x = (float)((double)sx / den);
        h.y = (float)((double)sy / den);
        const double num = walk ? (double)st * (1.0 / 65536.0) : 1.5625 * (double)st;
        h.tof_ns = (float)(num / den);
        h.npix = (uint32_t)cnt;
        h.shot = ev.shot[i];
        h.label = i;
        h.toa_first = q[5];
        h.tot_sum = (uint32_t)W;
        h.flags = W ? 0u : 1u;
        hits[k] = h;
    }
}
void launch_cent_emit(tpx_events ev, const uint32_t* order, uint64_t n_roots,
                      const uint64_t* acc, const uint64_t* trig, const float* walk,
                      tpx_hit* hits, uint64_t hit_cap, hipStream_t s) {
    if (n_roots)
        hipLaunchKernelGGL(k_cent_emit, dim3(grid_for(n_roots, 256, 4096)), dim3(256), 0, s, ev, order,
                           n_roots, acc, trig, walk, hits, hit_cap);
}

}  // namespace tpx
