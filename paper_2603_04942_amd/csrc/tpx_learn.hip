// Learned centroider / multiplicity splitter: 7 x 7 ToT/ToA patches of the
// clusters, and a 98 -> 256 -> 256 -> 8 MLP trained and run by the kernels
// below (bfloat16 operands on the matrix cores, fp32 accumulation).
//
// The patch of a hit is centred on the pixel nearest to its ToT-weighted
// centroid (Sec. V, Centroiding, Eq. 9); plane 0 holds the summed ToT of each
// pixel / 1024, plane 1 its earliest ToA minus the hit's earliest ToA in
// 64-tick (100 ns) units.  Outputs: two hits as corrections to the weighted
// centroid (x - xc, y - yc, (t - ToA_first) / 10 ns) and the logits of one and
// two hits; a network that outputs zeros reproduces the weighted centroid.
//
// Layout.  Parameters are one fp32 array packed W1[256][98], b1[256],
// W2[256][256], b2[256], W3[8][256], b3[8] (W as [out][in]).  Features are
// bfloat16 [n][98].  Every layer is one GEMM C = A * B with A(m, k) =
// A[m * sam + k * sak] and B(k, n) = B[k * sbk + n * sbn], so the transposed
// products of the backward pass need no transposed copies; the epilogue adds
// the bias, applies ReLU or the ReLU mask of the stored activation, and
// writes fp32 and/or bfloat16.
#include <type_traits>

#include "tpx_kernels.h"

namespace tpx {
namespace {

constexpr int kIn = 98, kHid = 256, kOut = 8, kCells = 49, kHalf = 3, kSide = 7;
constexpr size_t kOffW1 = 0, kOffB1 = kOffW1 + (size_t)kHid * kIn, kOffW2 = kOffB1 + kHid,
                 kOffB2 = kOffW2 + (size_t)kHid * kHid, kOffW3 = kOffB2 + kHid,
                 kOffB3 = kOffW3 + (size_t)kOut * kHid, kNParam = kOffB3 + kOut;
static_assert(kNParam == 93192, "parameter count of the 98-256-256-8 network");
constexpr size_t kFwdChunk = 65536;  // rows per forward pass in tpx_mlp_forward

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// gfx950's 16x16x32 bfloat16 MFMA: C[16][16] += A[16][32] B[32][16].  Lane
// l holds row (A) or column (B) l % 16 and eight k of group l / 16; any
// assignment of the 32 k to (group, element) gives the same product as long
// as A and B use the same one, and every caller here gives lane l the k
// 8 (l / 16) .. +7 in order.  Result lane l holds C[4 (l / 16) + r][l % 16],
// r = 0..3.
__device__ __forceinline__ f32x4 mfma32(s16x8 a, s16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// fp32 -> bfloat16, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// patch centre: x + 1/2 rounded down, in fp32
__device__ __forceinline__ int centre_of(float v) { return (int)floorf(v + 0.5f); }

// ------------------------------------------------------------------ patches
__global__ void k_patch_clear(uint32_t* acc, uint64_t n_hits) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_hits * kIn) return;
    acc[i] = (i % kIn) < kCells ? 0u : 0xFFFFFFFFu;
}

// one thread per event: find its hit by (shot, label) in the (shot, label)
// ordered hit list, then add its ToT and fold its ToA into the pixel's cell
// the hit of (shot, label) key in the (shot, label)-ordered hits: first
// index whose key is not below it
__device__ inline uint64_t hit_lower_bound(const tpx_hit* hits, uint64_t lo, uint64_t hi,
                                           uint64_t key) {
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        const uint64_t k = (hits[mid].shot << 32) | hits[mid].label;
        if (k < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One thread per event.  The events of a hit usually sit together, so the
// first active lane of the wave searches the whole hit list and every lane
// tries that hit and the next two before its own search.
__global__ void k_patch_accum(tpx_events ev, const uint32_t* labels, uint64_t n_ev,
                              const tpx_hit* hits, uint64_t n_hits, uint32_t* acc, int* err) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ev) return;
    const uint64_t key = ((uint64_t)ev.shot[i] << 32) | labels[i];
    const int first = __builtin_amdgcn_readfirstlane((int)__lane_id());
    const uint64_t lead_key = __shfl(key, first, 64);
    uint64_t lo = 0;
    if ((int)__lane_id() == first) lo = hit_lower_bound(hits, 0, n_hits, lead_key);
    const uint64_t guess = __shfl(lo, first, 64);
    bool found = false;
    for (uint64_t g = guess; g < guess + 3 && g < n_hits; ++g) {
        if (((hits[g].shot << 32) | hits[g].label) == key) {
            lo = g;
            found = true;
            break;
        }
    }
    if (!found) lo = hit_lower_bound(hits, 0, n_hits, key);
    if (lo >= n_hits || ((hits[lo].shot << 32) | hits[lo].label) != key) {
        atomicOr(err, 1);
        return;
    }
    const tpx_hit& h = hits[lo];
    const int ix = (int)ev.x[i] - centre_of(h.x) + kHalf;
    const int iy = (int)ev.y[i] - centre_of(h.y) + kHalf;
    if (ix < 0 || ix >= kSide || iy < 0 || iy >= kSide) return;
    const int c = iy * kSide + ix;
    const uint64_t toa = ev.toa[i];
    const uint64_t d = toa > h.toa_first ? toa - h.toa_first : 0;
    atomicAdd(&acc[lo * kIn + c], (uint32_t)ev.tot[i]);
    atomicMin(&acc[lo * kIn + kCells + c], d < 0xFFFFFFFEull ? (uint32_t)d : 0xFFFFFFFEu);
}

__global__ void k_patch_finish(const uint32_t* acc, uint64_t n_hits, uint16_t* feat) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_hits * kCells) return;
    const uint64_t h = i / kCells, c = i % kCells;
    const uint32_t s = acc[h * kIn + c];
    const uint32_t d = acc[h * kIn + kCells + c];
    feat[h * kIn + c] = to_bf16((float)(s < 1023u ? s : 1023u) * (1.0f / 1024.0f));
    feat[h * kIn + kCells + c] = d == 0xFFFFFFFFu ? (uint16_t)0 : to_bf16((float)d * (1.0f / 64.0f));
}

// Patches of the hits of a stream call, from its packed events (ToF ticks |
// ToT << 30 | y << 40 | x << 48), component ranks and segment offsets: the
// hit of an event is seg_off[segment] + rank.  Cells keep the smallest ToF;
// the hit's own smallest ToF (all its events, in the window or not) is the
// ToF of its toa_first, so cell - hit minimum = ToA - toa_first exactly.
__global__ void k_spatch_clear(uint32_t* acc, uint64_t n_hits) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_hits * (kIn + 1)) return;
    acc[i] = (i < n_hits * kIn && (i % kIn) < kCells) ? 0u : 0xFFFFFFFFu;
}

__global__ __launch_bounds__(256) void k_spatch_accum(ClusterArgs a, const tpx_hit* hits,
                                                      uint64_t n_hits, uint32_t* acc, int* err) {
    const uint64_t N = (a.skip && *a.skip) ? 0 : *a.n_ev_dev;
    const uint64_t n_seg = (N + a.q - 1) / a.q;
    const uint32_t k = blockIdx.x;
    if (k >= n_seg) return;
    const uint32_t g_lo = a.seg_lo[k], g_hi = a.seg_lo[k + 1];
    const uint64_t e0 = a.grp_off[g_lo], e1 = a.grp_off[g_hi];
    if (g_hi < g_lo || e1 < e0 || e1 > N) {
        if (threadIdx.x == 0) atomicOr(err, 1);
        return;
    }
    const uint32_t cnt = a.seg_cnt[k];
    const uint64_t out0 = a.seg_off[k];
    uint32_t* hmin = acc + n_hits * kIn;
    for (uint64_t p = e0 + threadIdx.x; p < e1; p += blockDim.x) {
        const uint32_t rk = a.rank[p];
        const uint64_t h = out0 + rk;
        if (rk >= cnt || h >= n_hits) {
            atomicOr(err, 1);
            continue;
        }
        const uint64_t pk = a.ev[p];
        const uint32_t tof = (uint32_t)(pk & 0x3FFFFFFFu);
        atomicMin(&hmin[h], tof);
        const int ix = (int)((pk >> 48) & 255u) - centre_of(hits[h].x) + kHalf;
        const int iy = (int)((pk >> 40) & 255u) - centre_of(hits[h].y) + kHalf;
        if (ix < 0 || ix >= kSide || iy < 0 || iy >= kSide) continue;
        const int c = iy * kSide + ix;
        atomicAdd(&acc[h * kIn + c], (uint32_t)((pk >> 30) & 1023u));
        atomicMin(&acc[h * kIn + kCells + c], tof);
    }
}

// the same from the hit of every event recorded by the fused kernel
__global__ __launch_bounds__(256) void k_spatch_accum_idx(ClusterArgs a, const tpx_hit* hits,
                                                          uint64_t n_hits, uint32_t* acc, int* err) {
    const uint64_t N = (a.skip && *a.skip) ? 0 : *a.n_ev_dev;
    uint32_t* hmin = acc + n_hits * kIn;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t h = a.hit_index[p];
        if (h >= n_hits) {
            atomicOr(err, 1);
            continue;
        }
        const uint64_t pk = a.ev[p];
        const uint32_t tof = (uint32_t)(pk & 0x3FFFFFFFu);
        atomicMin(&hmin[h], tof);
        const int ix = (int)((pk >> 48) & 255u) - centre_of(hits[h].x) + kHalf;
        const int iy = (int)((pk >> 40) & 255u) - centre_of(hits[h].y) + kHalf;
        if (ix < 0 || ix >= kSide || iy < 0 || iy >= kSide) continue;
        const int c = iy * kSide + ix;
        atomicAdd(&acc[h * kIn + c], (uint32_t)((pk >> 30) & 1023u));
        atomicMin(&acc[h * kIn + kCells + c], tof);
    }
}

__global__ void k_spatch_finish(const uint32_t* acc, uint64_t n_hits, uint16_t* feat) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_hits * kCells) return;
    const uint64_t h = i / kCells, c = i % kCells;
    const uint32_t s = acc[h * kIn + c];
    const uint32_t d = acc[h * kIn + kCells + c];
    const uint32_t m = acc[n_hits * kIn + h];
    feat[h * kIn + c] = to_bf16((float)(s < 1023u ? s : 1023u) * (1.0f / 1024.0f));
    feat[h * kIn + kCells + c] =
        d == 0xFFFFFFFFu ? (uint16_t)0 : to_bf16((float)(d - m) * (1.0f / 64.0f));
}

// --------------------------------------------------------------------- GEMM
struct Gemm {
    const uint16_t* A;
    int64_t sam, sak;
    const uint16_t* B;
    int64_t sbk, sbn;
    int M, N, K;
    const float* bias;      // [N] or null
    int relu;
    const uint16_t* mask;   // keep (m, n) only where mask[m * ldmask + n] > 0, or null
    int64_t ldmask;
    float* C32;             // or null
    int64_t ldc32;
    uint16_t* C16;          // or null
    int64_t ldc16;
    int k_chunk;            // k per workgroup along z (split-K); K when not split
    int64_t split_stride;   // C32 offset between the z slices
};

constexpr int kTM = 64, kTK = 32, kPitch = kTK + 8;

// Loads a rows x 32 tile of a strided operand into LDS as [row][k].  When k
// is contiguous (stride 1) and K is a multiple of the vector width, each
// thread moves `vec` consecutive k at once (a vector of 2 or 4 bfloat16);
// otherwise one element at a time, with consecutive threads along whichever
// of row / k is contiguous.
// One rows x 32 tile of a strided operand, moved in two halves so that the
// next tile's global loads are in flight while the current one is multiplied:
// fetch() issues the loads into registers, stash() writes them to LDS as
// [row][k].  When k is contiguous (stride 1) and K is a multiple of the
// vector width, each thread moves `vec` consecutive k at once (a vector of 2
// or 4 bfloat16); otherwise one element at a time, with consecutive threads
// along whichever of row / k is contiguous.  Trip counts are compile-time
// constants (rows * 32 / vec is a multiple of 256).
template <int kRows, int vec>
struct TileRegs {
    static_assert((kRows * kTK / 4) % 256 == 0, "tile rows must be a multiple of 32");
    static constexpr int kN = kRows * kTK / vec / 256;
    using V = typename std::conditional<vec == 4, uint2,
                                        typename std::conditional<vec == 2, uint32_t,
                                                                  uint16_t>::type>::type;
    V v[kN];

    __device__ __forceinline__ static void pos(int e, bool k_contig, int* r, int* k) {
        if constexpr (vec == 4) {
            *r = e >> 3, *k = (e & 7) * 4;
        } else if constexpr (vec == 2) {
            *r = e >> 4, *k = (e & 15) * 2;
        } else {
            *r = k_contig ? e >> 5 : e % kRows;
            *k = k_contig ? e & 31 : e / kRows;
        }
    }

    __device__ __forceinline__ void fetch(const uint16_t* src, int64_t s_row, int64_t s_k,
                                          int row0, int n_rows, int k0, int K, int tid) {
        const bool k_contig = s_k == 1;
#pragma unroll
        for (int it = 0; it < kN; ++it) {
            int r, k;
            pos(tid + 256 * it, k_contig, &r, &k);
            const int gr = row0 + r, gk = k0 + k;
            const bool in = gr < n_rows && gk < K;
            if constexpr (vec == 4) {
                v[it] = in ? *(const uint2*)(src + gr * s_row + gk) : make_uint2(0u, 0u);
            } else if constexpr (vec == 2) {
                v[it] = in ? *(const uint32_t*)(src + gr * s_row + gk) : 0u;
            } else {
                v[it] = in ? src[gr * s_row + gk * s_k] : (uint16_t)0;
            }
        }
    }

    __device__ __forceinline__ void stash(uint16_t (*T)[kPitch], int64_t s_k, int tid) const {
        const bool k_contig = s_k == 1;
#pragma unroll
        for (int it = 0; it < kN; ++it) {
            int r, k;
            pos(tid + 256 * it, k_contig, &r, &k);
            *(V*)&T[r][k] = v[it];
        }
    }
};

// vector width for a k-contiguous operand: every row start and K aligned
__host__ inline int vec_width(const uint16_t* p, int64_t s_row, int64_t s_k, int K) {
    if (s_k != 1) return 1;
    const uintptr_t a = (uintptr_t)p;
    if (K % 4 == 0 && s_row % 4 == 0 && a % 8 == 0) return 4;
    if (K % 2 == 0 && s_row % 2 == 0 && a % 4 == 0) return 2;
    return 1;
}

// 256 threads = 4 waves in 2 x 2; each wave owns a 32 x (kTN / 2) block of
// the 64 x kTN tile as 2 x (kTN / 32) MFMA 16x16x32 blocks (one MFMA per
// block and 32-deep k-step).
template <int kTN, int kVA, int kVB>
__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
    constexpr int kNB = kTN / 32;
    __shared__ __align__(16) uint16_t As[kTM][kPitch];
    __shared__ __align__(16) uint16_t Bs[kTN][kPitch];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    f32x4 acc[2][kNB];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < kNB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    TileRegs<kTM, kVA> ra;
    TileRegs<kTN, kVB> rb;
    // this workgroup's range of k (all of it unless split along z)
    const int kb = (int)blockIdx.z * g.k_chunk;
    const int ke = g.K < kb + g.k_chunk ? g.K : kb + g.k_chunk;
    ra.fetch(g.A, g.sam, g.sak, m0, g.M, kb, ke, tid);
    rb.fetch(g.B, g.sbn, g.sbk, n0, g.N, kb, ke, tid);
    for (int k0 = kb; k0 < ke; k0 += kTK) {
        ra.stash(As, g.sak, tid);
        rb.stash(Bs, g.sbk, tid);
        __syncthreads();
        if (k0 + kTK < ke) {  // the next tile's loads overlap this tile's products
            ra.fetch(g.A, g.sam, g.sak, m0, g.M, k0 + kTK, ke, tid);
            rb.fetch(g.B, g.sbn, g.sbk, n0, g.N, k0 + kTK, ke, tid);
        }
        static_assert(kTK == 32, "one 16x16x32 MFMA per block and k-step");
        {
            s16x8 a[2], b[kNB];
            const int kq = 8 * (lane >> 4);
            for (int mb = 0; mb < 2; ++mb)
                a[mb] = *(const s16x8*)&As[wm * 32 + mb * 16 + (lane & 15)][kq];
            for (int nb = 0; nb < kNB; ++nb)
                b[nb] = *(const s16x8*)&Bs[wn * (kTN / 2) + nb * 16 + (lane & 15)][kq];
            for (int mb = 0; mb < 2; ++mb)
                for (int nb = 0; nb < kNB; ++nb) acc[mb][nb] = mfma32(a[mb], b[nb], acc[mb][nb]);
        }
        __syncthreads();
    }
    for (int mb = 0; mb < 2; ++mb)
        for (int nb = 0; nb < kNB; ++nb)
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * 32 + mb * 16 + 4 * (lane >> 4) + r;
                const int n = n0 + wn * (kTN / 2) + nb * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[mb][nb][r];
                if (g.bias) v += g.bias[n];
                if (g.relu) v = v > 0.f ? v : 0.f;
                if (g.mask && !(from_bf16(g.mask[m * g.ldmask + n]) > 0.f)) v = 0.f;
                if (g.C32) g.C32[blockIdx.z * g.split_stride + m * g.ldc32 + n] = v;
                if (g.C16) g.C16[m * g.ldc16 + n] = to_bf16(v);
            }
}

// k per slice when k is split `splits` ways (a multiple of the tile depth),
// and the number of slices that then cover K
inline int split_chunk(int K, int splits) {
    const int c = (((K + splits - 1) / splits + kTK - 1) / kTK) * kTK;
    return c < kTK ? kTK : c;
}
inline int split_count(int K, int chunk) {
    const int n = (K + chunk - 1) / chunk;
    return n < 1 ? 1 : n;
}

void gemm(Gemm g, hipStream_t s, int splits = 1) {
    if (g.M <= 0 || g.N <= 0) return;
    // split-K slices are partial sums: an epilogue (bias, ReLU, mask, the
    // bfloat16 copy) applies only to a whole sum, so such products run unsplit
    if (g.bias || g.relu || g.mask || g.C16) splits = 1;
    g.k_chunk = split_chunk(g.K, splits);
    splits = split_count(g.K, g.k_chunk);
    // 64 x 64 tiles: the weight-gradient products (M, N <= 256, K = batch)
    // need every workgroup they can get; a 128-wide tile measured no faster
    // on the forward products either
    // one instantiation per pair of operand vector widths, so that each
    // kernel holds only its own load path (registers, occupancy)
    const int va = vec_width(g.A, g.sam, g.sak, g.K), vb = vec_width(g.B, g.sbn, g.sbk, g.K);
    dim3 grid((g.N + 63) / 64, (g.M + kTM - 1) / kTM, splits);
#define TPX_GEMM(A_, B_)                                                      \
    if (va == A_ && vb == B_) {                                               \
        hipLaunchKernelGGL((k_gemm<64, A_, B_>), grid, dim3(256), 0, s, g); \
        return;                                                               \
    }
    TPX_GEMM(1, 1) TPX_GEMM(1, 2) TPX_GEMM(1, 4)
    TPX_GEMM(2, 1) TPX_GEMM(2, 2) TPX_GEMM(2, 4)
    TPX_GEMM(4, 1) TPX_GEMM(4, 2) TPX_GEMM(4, 4)
#undef TPX_GEMM
}

// sums the z slices of a split-K product in slice order (deterministic)
__global__ void k_sum_splits(const float* part, int splits, int M, int N, float* C, int64_t ldc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * N) return;
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += part[(int64_t)z * M * N + i];
    C[(int64_t)(i / N) * ldc + i % N] = v;
}

constexpr int kMaxSplits = 16;

// A weight-gradient product (M, N <= 256, K = batch, plain fp32 output): few
// output tiles and a long k, so k is split over up to 16 workgroups per tile
// into `part` (kMaxSplits * M * N floats) and the slices summed in order.
void gemm_wgrad(const Gemm& g, float* part, hipStream_t s) {
    const int tiles = ((g.N + 63) / 64) * ((g.M + kTM - 1) / kTM);
    int splits = g.K / 256;
    if (splits > kMaxSplits) splits = kMaxSplits;
    if (tiles >= 64 || splits < 2) {
        gemm(g, s);
        return;
    }
    Gemm h = g;
    h.C32 = part, h.ldc32 = g.N, h.split_stride = (int64_t)g.M * g.N;
    gemm(h, s, splits);
    const int used = split_count(g.K, split_chunk(g.K, splits));
    hipLaunchKernelGGL(k_sum_splits, dim3((g.M * g.N + 255) / 256), dim3(256), 0, s, part, used,
                       g.M, g.N, g.C32, g.ldc32);
}

// ------------------------------------------------------- loss, sums, update
__global__ void k_cast_bf16(const float* p, uint64_t n, uint16_t* q) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = to_bf16(p[i]);
}

__global__ void k_zero_f32(float* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0.f;
}

// one thread per sample: targets relative to the weighted centroid and the
// earliest ToA, the loss (pair matched the cheaper way round, ties A-first), dL/dO / n
__global__ void k_loss(const float* O, const tpx_hit* hits, const float* truth,
                       const uint8_t* mult, int n, float* G32, uint16_t* G16, float* loss_sum) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float li = 0.f;
    if (i < n) {
        const tpx_hit& h = hits[i];
        const double t0 = (double)h.toa_first * 1.5625;
        float T[2][3];
        for (int k = 0; k < 2; ++k) {
            T[k][0] = truth[i * 6 + 3 * k + 0] - h.x;
            T[k][1] = truth[i * 6 + 3 * k + 1] - h.y;
            T[k][2] = (float)(((double)truth[i * 6 + 3 * k + 2] - t0) / 10.0);
        }
        float o[8];
        for (int k = 0; k < 8; ++k) o[k] = O[i * 8 + k];
        const bool two = mult[i] == 2;
        float ea = 0.f, c1b = 0.f, c2 = 0.f;
        for (int k = 0; k < 3; ++k) {
            ea += (o[k] - T[0][k]) * (o[k] - T[0][k]);
            c1b += (o[3 + k] - T[1][k]) * (o[3 + k] - T[1][k]);
            c2 += (o[k] - T[1][k]) * (o[k] - T[1][k]) + (o[3 + k] - T[0][k]) * (o[3 + k] - T[0][k]);
        }
        const float c1 = ea + c1b;
        const bool swap = two && c2 < c1;
        const float lpos = two ? fminf(c1, c2) : ea;
        const float mx = fmaxf(o[6], o[7]);
        const float lse = mx + logf(expf(o[6] - mx) + expf(o[7] - mx));
        li = lpos + lse - (two ? o[7] : o[6]);
        const float inv = 1.0f / (float)n;
        float g[8];
        for (int k = 0; k < 3; ++k) {
            g[k] = 2.f * (o[k] - (swap ? T[1][k] : T[0][k])) * inv;
            g[3 + k] = two ? 2.f * (o[3 + k] - (swap ? T[0][k] : T[1][k])) * inv : 0.f;
        }
        const float p1 = expf(o[6] - lse), p2 = expf(o[7] - lse);
        g[6] = (p1 - (two ? 0.f : 1.f)) * inv;
        g[7] = (p2 - (two ? 1.f : 0.f)) * inv;
        for (int k = 0; k < 8; ++k) {
            G32[i * 8 + k] = g[k];
            G16[i * 8 + k] = to_bf16(g[k]);
        }
    }
    // block sum of the sample losses, one atomic per block
    __shared__ float part[4];
    float v = li;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss_sum, part[0] + part[1] + part[2] + part[3]);
}

// column sums of an fp32 [rows][cols] matrix: one workgroup per column
__global__ void k_colsum(const float* a, int rows, int cols, float* out) {
    const int c = blockIdx.x;
    float v = 0.f;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) v += a[(int64_t)r * cols + c];
    __shared__ float part[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[c] = part[0] + part[1] + part[2] + part[3];
}

__global__ void k_adam(float* p, float* m, float* v, const float* g, uint64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_refine(const tpx_hit* hits, const float* O, uint64_t n, float* out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const tpx_hit& h = hits[i];
    const double t0 = (double)h.toa_first * 1.5625;
    const float p2 = 1.f / (1.f + expf(O[i * 8 + 6] - O[i * 8 + 7]));
    // a cluster judged single (logit of two not above that of one) keeps the
    // weighted centroid's position
    const float keep = O[i * 8 + 7] > O[i * 8 + 6] ? 1.f : 0.f;
    for (int k = 0; k < 2; ++k) {
        out[i * 8 + 3 * k + 0] = h.x + keep * O[i * 8 + 3 * k + 0];
        out[i * 8 + 3 * k + 1] = h.y + keep * O[i * 8 + 3 * k + 1];
        out[i * 8 + 3 * k + 2] = (float)(t0 + 10.0 * (double)O[i * 8 + 3 * k + 2]);
    }
    out[i * 8 + 6] = p2;
    out[i * 8 + 7] = 0.f;
}

inline unsigned blocks(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// workspace of one pass over `rows` samples
struct MlpWs {
    uint16_t *wq, *h1, *h2, *g16, *z2_16, *z1_16;
    float *o, *g32, *z2_32, *z1_32, *loss, *part;
};

size_t mlp_ws_bytes(size_t rows) {
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return r(kNParam * 2) + 2 * r(rows * kHid * 2) + r(rows * kOut * 2) + 2 * r(rows * kHid * 2) +
           r(rows * kOut * 4) + r(rows * kOut * 4) + 2 * r(rows * kHid * 4) + r(64) +
           r((size_t)kMaxSplits * kHid * kHid * 4);
}

MlpWs carve_mlp(void* ws, size_t rows) {
    uintptr_t p = (uintptr_t)ws;
    auto take = [&](size_t b) {
        const uintptr_t q = p;
        p += (b + 255) & ~(size_t)255;
        return (void*)q;
    };
    MlpWs w;
    w.wq = (uint16_t*)take(kNParam * 2);
    w.h1 = (uint16_t*)take(rows * kHid * 2);
    w.h2 = (uint16_t*)take(rows * kHid * 2);
    w.g16 = (uint16_t*)take(rows * kOut * 2);
    w.z2_16 = (uint16_t*)take(rows * kHid * 2);
    w.z1_16 = (uint16_t*)take(rows * kHid * 2);
    w.o = (float*)take(rows * kOut * 4);
    w.g32 = (float*)take(rows * kOut * 4);
    w.z2_32 = (float*)take(rows * kHid * 4);
    w.z1_32 = (float*)take(rows * kHid * 4);
    w.loss = (float*)take(64);
    w.part = (float*)take((size_t)kMaxSplits * kHid * kHid * 4);
    return w;
}

Gemm mk(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk, int64_t sbn,
        int M, int N, int K) {
    Gemm g{};
    g.A = A, g.sam = sam, g.sak = sak, g.B = B, g.sbk = sbk, g.sbn = sbn;
    g.M = M, g.N = N, g.K = K;
    return g;
}

// forward of `rows` samples from feat into o (fp32 [rows][8]); wq holds the
// bfloat16 weights; h1, h2 keep the bfloat16 activations for the backward
void forward(const float* params, const uint16_t* wq, const uint16_t* feat, int rows, uint16_t* h1,
             uint16_t* h2, float* o, hipStream_t s) {
    Gemm g = mk(feat, kIn, 1, wq + kOffW1, 1, kIn, rows, kHid, kIn);
    g.bias = params + kOffB1, g.relu = 1, g.C16 = h1, g.ldc16 = kHid;
    gemm(g, s);
    g = mk(h1, kHid, 1, wq + kOffW2, 1, kHid, rows, kHid, kHid);
    g.bias = params + kOffB2, g.relu = 1, g.C16 = h2, g.ldc16 = kHid;
    gemm(g, s);
    g = mk(h2, kHid, 1, wq + kOffW3, 1, kHid, rows, kOut, kHid);
    g.bias = params + kOffB3, g.C32 = o, g.ldc32 = kOut;
    gemm(g, s);
}

// ------------------------------------------------------ fused forward pass
// Inference only: one workgroup per 64 rows runs all three layers with the
// input tile and both hidden activations in LDS (no hidden activations in
// HBM); weights come from L2 straight into the MFMA operand registers, the
// next k-step's prefetched.  Same products in the same order and the same
// epilogue rounding as the layered GEMMs.
constexpr int kFR = 64, kXK = 128, kXP = kXK + 8, kHP = kHid + 8;
static_assert(kXK % 32 == 0 && kXK >= kIn, "layer-1 k padded to whole 32-deep steps");

// eight consecutive bfloat16 weights (p 4-byte aligned; 16-byte loads when
// the rows allow)
__device__ __forceinline__ s16x8 load_w8(const uint16_t* p, bool aligned16) {
    if (aligned16) return *(const s16x8*)p;
    const uint4 t = make_uint4(*(const uint32_t*)p, *(const uint32_t*)(p + 2),
                               *(const uint32_t*)(p + 4), *(const uint32_t*)(p + 6));
    return __builtin_bit_cast(s16x8, t);
}

// Out[64][256] = relu(A[64][K] W^T + bias) in bfloat16; wave w computes
// columns [64 w, 64 w + 64) as 4 x 4 MFMA blocks.  W rows are `ldw` apart;
// operand k beyond a row's end meets zeros of A (the padding of layer 1).
template <int K, int P>
__device__ __forceinline__ void dense_relu(const uint16_t (*A)[P], const uint16_t* W, int ldw,
                                           const float* bias, uint16_t (*Out)[kHP], int w,
                                           int lane) {
    const int j = lane & 15, kq = 8 * (lane >> 4);
    const bool al = (ldw % 8) == 0;
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    s16x8 bc[4], bn[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) bc[nb] = load_w8(W + (int64_t)(w * 64 + nb * 16 + j) * ldw + kq, al);
    for (int k0 = 0; k0 < K; k0 += 32) {
        if (k0 + 32 < K) {
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                bn[nb] = load_w8(W + (int64_t)(w * 64 + nb * 16 + j) * ldw + k0 + 32 + kq, al);
        }
        s16x8 a[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) a[mb] = *(const s16x8*)&A[mb * 16 + j][k0 + kq];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = mfma32(a[mb], bc[nb], acc[mb][nb]);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) bc[nb] = bn[nb];
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = mb * 16 + 4 * (lane >> 4) + r, col = w * 64 + nb * 16 + j;
                float v = acc[mb][nb][r] + bias[col];
                Out[row][col] = to_bf16(v > 0.f ? v : 0.f);
            }
}

__global__ __launch_bounds__(256, 2) void k_mlp_fused(const float* __restrict__ params,
                                                      const uint16_t* __restrict__ wq,
                                                      const uint16_t* __restrict__ feat, int n,
                                                      float* __restrict__ out) {
    __shared__ __align__(16) uint16_t H1[kFR][kHP];
    __shared__ __align__(16) uint16_t XB[kFR * kHP];  // X [64][kXP] in layer 1, then H2 [64][kHP]
    uint16_t(*X)[kXP] = (uint16_t(*)[kXP])XB;
    uint16_t(*H2)[kHP] = (uint16_t(*)[kHP])XB;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r0 = blockIdx.x * kFR;
    // input tile, zero beyond the 98 features and the last row
    for (int e = tid; e < kFR * (kXK / 2); e += 256) {
        const int r = e / (kXK / 2), c = 2 * (e % (kXK / 2));
        uint32_t v = 0u;
        if (r0 + r < n && c < kIn) v = *(const uint32_t*)(feat + (int64_t)(r0 + r) * kIn + c);
        *(uint32_t*)&X[r][c] = v;
    }
    __syncthreads();
    dense_relu<kXK, kXP>(X, wq + kOffW1, kIn, params + kOffB1, H1, w, lane);
    __syncthreads();
    dense_relu<kHid, kHP>(H1, wq + kOffW2, kHid, params + kOffB2, H2, w, lane);
    __syncthreads();
    // output layer: wave w takes rows [16 w, 16 w + 16), columns 0..7 of a
    // 16-wide MFMA block
    const int j = lane & 15, kq = 8 * (lane >> 4);
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < kHid; k0 += 32) {
        const s16x8 a = *(const s16x8*)&H2[w * 16 + j][k0 + kq];
        s16x8 b = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
        if (j < kOut) b = *(const s16x8*)(wq + kOffW3 + j * kHid + k0 + kq);
        acc = mfma32(a, b, acc);
    }
    if (j < kOut) {
        const float b3 = params[kOffB3 + j];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = r0 + w * 16 + 4 * (lane >> 4) + r;
            if (row < n) out[(int64_t)row * kOut + j] = acc[r] + b3;
        }
    }
}

}  // namespace

void launch_stream_patches(const ClusterArgs& a, uint64_t grid, bool fused, const tpx_hit* hits,
                           uint64_t n_hits, uint32_t* acc, uint16_t* feat, int* err,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, (float*)err, 1);
    hipLaunchKernelGGL(k_spatch_clear, dim3(blocks(n_hits * (kIn + 1), 256)), dim3(256), 0, s,
                       acc, n_hits);
    if (fused)
        hipLaunchKernelGGL(k_spatch_accum_idx, dim3(2048), dim3(256), 0, s, a, hits, n_hits, acc,
                           err);
    else if (grid)
        hipLaunchKernelGGL(k_spatch_accum, dim3((unsigned)grid), dim3(256), 0, s, a, hits, n_hits,
                           acc, err);
    hipLaunchKernelGGL(k_spatch_finish, dim3(blocks(n_hits * kCells, 256)), dim3(256), 0, s, acc,
                       n_hits, feat);
}

}  // namespace tpx

using namespace tpx;

extern "C" {

size_t tpx_patch_workspace_bytes(size_t n_hits) { return n_hits * kIn * 4 + 256; }

tpx_status tpx_patches(tpx_events ev, const uint32_t* labels, size_t n_ev, const tpx_hit* hits,
                       size_t n_hits, uint16_t* feat, void* ws, size_t ws_bytes, void* stream) {
    if (n_ev && (!ev.x || !ev.y || !ev.tot || !ev.shot || !ev.toa || !labels))
        return report(TPX_EINVAL, "an event array is NULL");
    if (n_hits && (!hits || !feat)) return report(TPX_EINVAL, "hits or feat is NULL");
    if (n_ev && !n_hits) return report(TPX_EINVAL, "events without hits");
    if (!ws || ws_bytes < tpx_patch_workspace_bytes(n_hits))
        return report(TPX_EINVAL, "workspace too small");
    if (n_hits == 0) return TPX_OK;
    hipStream_t s = (hipStream_t)stream;
    uint32_t* acc = (uint32_t*)ws;
    int* err = (int*)((char*)ws + n_hits * kIn * 4);
    hipLaunchKernelGGL(k_patch_clear, dim3(blocks(n_hits * kIn, 256)), dim3(256), 0, s, acc,
                       (uint64_t)n_hits);
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, (float*)err, 1);
    if (n_ev)
        hipLaunchKernelGGL(k_patch_accum, dim3(blocks(n_ev, 256)), dim3(256), 0, s, ev, labels,
                           (uint64_t)n_ev, hits, (uint64_t)n_hits, acc, err);
    hipLaunchKernelGGL(k_patch_finish, dim3(blocks(n_hits * kCells, 256)), dim3(256), 0, s, acc,
                       (uint64_t)n_hits, feat);
    int e = 0;
    if (hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return report(TPX_EHIP, "patch kernels failed");
    if (e) return report(TPX_EINVAL, "an event's (shot, label) has no hit");
    return TPX_OK;
}

size_t tpx_mlp_workspace_bytes(size_t batch) { return mlp_ws_bytes(batch); }

tpx_status tpx_mlp_forward(const float* params, const uint16_t* feat, size_t n, float* out,
                           void* ws, size_t ws_bytes, void* stream) {
    if (n && (!params || !feat || !out)) return report(TPX_EINVAL, "NULL argument");
    const size_t rows = n < kFwdChunk ? n : kFwdChunk;
    if (!ws || ws_bytes < mlp_ws_bytes(rows)) return report(TPX_EINVAL, "workspace too small");
    if (n == 0) return TPX_OK;
    hipStream_t s = (hipStream_t)stream;
    MlpWs w = carve_mlp(ws, rows);
    hipLaunchKernelGGL(k_cast_bf16, dim3(blocks(kNParam, 256)), dim3(256), 0, s, params,
                       (uint64_t)kNParam, w.wq);
    for (size_t r0 = 0; r0 < n; r0 += rows) {
        const int m = (int)(n - r0 < rows ? n - r0 : rows);
        hipLaunchKernelGGL(k_mlp_fused, dim3(blocks((uint64_t)m, kFR)), dim3(256), 0, s, params,
                           w.wq, feat + r0 * kIn, m, out + r0 * kOut);
    }
    if (hipGetLastError() != hipSuccess) return report(TPX_EHIP, "forward launch failed");
    return TPX_OK;
}

tpx_status tpx_mlp_grad(const float* params, const uint16_t* feat, const tpx_hit* hits,
                        const float* truth, const uint8_t* mult, size_t n, float* grad,
                        float* loss_h, void* ws, size_t ws_bytes, void* stream) {
    if (!params || !grad || (n && (!feat || !hits || !truth || !mult)))
        return report(TPX_EINVAL, "NULL argument");
    if (n == 0 || n > (1u << 24)) return report(TPX_EINVAL, "batch size out of range");
    if (!ws || ws_bytes < mlp_ws_bytes(n)) return report(TPX_EINVAL, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int B = (int)n;
    MlpWs w = carve_mlp(ws, n);
    hipLaunchKernelGGL(k_cast_bf16, dim3(blocks(kNParam, 256)), dim3(256), 0, s, params,
                       (uint64_t)kNParam, w.wq);
    forward(params, w.wq, feat, B, w.h1, w.h2, w.o, s);
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, w.loss, 1);
    hipLaunchKernelGGL(k_loss, dim3(blocks(n, 256)), dim3(256), 0, s, w.o, hits, truth, mult, B,
                       w.g32, w.g16, w.loss);
    // layer 3: dW3 = G^T H2, db3 = sum G, dZ2 = (G W3) * [H2 > 0]
    Gemm g = mk(w.g16, 1, kOut, w.h2, kHid, 1, kOut, kHid, B);
    g.C32 = grad + kOffW3, g.ldc32 = kHid;
    gemm_wgrad(g, w.part, s);
    hipLaunchKernelGGL(k_colsum, dim3(kOut), dim3(256), 0, s, w.g32, B, kOut, grad + kOffB3);
    g = mk(w.g16, kOut, 1, w.wq + kOffW3, kHid, 1, B, kHid, kOut);
    g.mask = w.h2, g.ldmask = kHid, g.C32 = w.z2_32, g.ldc32 = kHid, g.C16 = w.z2_16, g.ldc16 = kHid;
    gemm(g, s);
    // layer 2: dW2 = dZ2^T H1, db2 = sum dZ2, dZ1 = (dZ2 W2) * [H1 > 0]
    g = mk(w.z2_16, 1, kHid, w.h1, kHid, 1, kHid, kHid, B);
    g.C32 = grad + kOffW2, g.ldc32 = kHid;
    gemm_wgrad(g, w.part, s);
    hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, w.z2_32, B, kHid, grad + kOffB2);
    g = mk(w.z2_16, kHid, 1, w.wq + kOffW2, kHid, 1, B, kHid, kHid);
    g.mask = w.h1, g.ldmask = kHid, g.C32 = w.z1_32, g.ldc32 = kHid, g.C16 = w.z1_16, g.ldc16 = kHid;
    gemm(g, s);
    // layer 1: dW1 = dZ1^T X, db1 = sum dZ1
    g = mk(w.z1_16, 1, kHid, feat, kIn, 1, kHid, kIn, B);
    g.C32 = grad + kOffW1, g.ldc32 = kIn;
    gemm_wgrad(g, w.part, s);
    hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, w.z1_32, B, kHid, grad + kOffB1);
    if (hipGetLastError() != hipSuccess) return report(TPX_EHIP, "gradient launch failed");
    if (loss_h) {
        float l = 0.f;
        if (hipMemcpyAsync(&l, w.loss, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return report(TPX_EHIP, "loss copy failed");
        *loss_h = l / (float)n;
    }
    return TPX_OK;
}

tpx_status tpx_mlp_adam(float* params, float* m, float* v, const float* grad, size_t n_param,
                        uint64_t step, float lr, float beta1, float beta2, float eps,
                        void* stream) {
    if (!params || !m || !v || !grad) return report(TPX_EINVAL, "NULL argument");
    if (step == 0) return report(TPX_EINVAL, "step counts from 1");
    const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
    hipLaunchKernelGGL(k_adam, dim3(blocks(n_param, 256)), dim3(256), 0, (hipStream_t)stream,
                       params, m, v, grad, (uint64_t)n_param, lr, beta1, beta2, eps, c1, c2);
    if (hipGetLastError() != hipSuccess) return report(TPX_EHIP, "adam launch failed");
    return TPX_OK;
}

tpx_status tpx_mlp_refine(const tpx_hit* hits, const float* out, size_t n, float* refined,
                          void* stream) {
    if (n && (!hits || !out || !refined)) return report(TPX_EINVAL, "NULL argument");
    if (n == 0) return TPX_OK;
    hipLaunchKernelGGL(k_refine, dim3(blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, hits,
                       out, (uint64_t)n, refined);
    if (hipGetLastError() != hipSuccess) return report(TPX_EHIP, "refine launch failed");
    return TPX_OK;
}

}  // extern "C"
