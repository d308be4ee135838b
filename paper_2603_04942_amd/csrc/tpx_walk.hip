// Walk calibration (Sec. IV, ToT-ToF Correlation Correction, Eq. 1).
//
// A calibration run holds hits of one ion species; the pixels of its peak
// (ToF in a narrow window) reach the detector at one true time, and their
// measured ToF drifts later as ToT falls (time walk).  For every ToT value
// the centre of its ToF distribution is taken (the Gaussian's
// maximum-likelihood centre: the mean ToF of the slice's pixels of that
// ToT), and Eq. (1), a / (ToT + b)^d + c, is fitted to the centres by least
// squares weighted by the pixel counts (the same minimum as a fit over the
// individual pixels).  The data-parallel part, the per-ToT counts and ToF
// sums of millions of pixels, runs in k_walk_bins (per-workgroup LDS bins,
// exact integer sums); the four-parameter Levenberg-Marquardt fit over at
// most 1,024 centres runs on the host.
#include <cmath>
#include <cstdio>
#include <vector>

#include "tpx_kernels.h"

namespace tpx {
namespace {

constexpr int kBins = 1024;
constexpr int kWalkWG = 256;
constexpr int kWalkBlocks = 512;

// bins[t] = pixel count, bins[kBins + t] = sum of (ToF - tof_lo) in ticks, of
// the pixels of ToT t with tof_lo <= ToF <= tof_hi; bins[2 kBins] = events
// whose shot has no trigger time.
__global__ __launch_bounds__(kWalkWG) void k_walk_bins(tpx_events ev, uint64_t n,
                                                       const uint64_t* __restrict__ trig,
                                                       uint64_t n_trig, uint64_t lo, uint64_t hi,
                                                       unsigned long long* bins) {
    __shared__ uint32_t cnt[kBins];
    __shared__ unsigned long long sum[kBins];
    for (int t = threadIdx.x; t < kBins; t += kWalkWG) {
        cnt[t] = 0;
        sum[t] = 0;
    }
    __syncthreads();
    unsigned long long bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kWalkWG + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kWalkWG) {
        const uint32_t s = ev.shot[i];
        if (s >= n_trig) {
            ++bad;
            continue;
        }
        const uint64_t toa = ev.toa[i], t0 = trig[s];
        if (toa < t0) continue;
        const uint64_t tof = toa - t0;
        if (tof < lo || tof > hi) continue;
        const uint32_t tot = ev.tot[i] & 1023u;
        atomicAdd(&cnt[tot], 1u);
        atomicAdd(&sum[tot], (unsigned long long)(tof - lo));
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kBins; t += kWalkWG) {
        if (cnt[t]) {
            atomicAdd(&bins[t], (unsigned long long)cnt[t]);
            atomicAdd(&bins[kBins + t], sum[t]);
        }
    }
    if (bad) atomicAdd(&bins[2 * kBins], bad);
}

__global__ void k_walk_clear(unsigned long long* bins) {
    for (int i = threadIdx.x; i < 2 * kBins + 1; i += blockDim.x) bins[i] = 0;
}

// Eq. (1) and its partial derivatives in (a, b, d, c)
inline double model(double t, const double* p) { return p[0] / std::pow(t + p[1], p[2]) + p[3]; }
inline void grad(double t, const double* p, double* g) {
    const double u = std::pow(t + p[1], -p[2]);
    g[0] = u;
    g[1] = -p[0] * p[2] * u / (t + p[1]);
    g[2] = -p[0] * u * std::log(t + p[1]);
    g[3] = 1.0;
}

// solves the 4x4 system m x = v (Gaussian elimination with partial pivoting);
// false when singular
bool solve4(double m[4][4], double v[4], double x[4]) {
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (std::fabs(m[r][c]) > std::fabs(m[piv][c])) piv = r;
        if (m[piv][c] == 0.0 || !std::isfinite(m[piv][c])) return false;
        if (piv != c) {
            for (int k = 0; k < 4; ++k) std::swap(m[c][k], m[piv][k]);
            std::swap(v[c], v[piv]);
        }
        for (int r = c + 1; r < 4; ++r) {
            const double f = m[r][c] / m[c][c];
            for (int k = c; k < 4; ++k) m[r][k] -= f * m[c][k];
            v[r] -= f * v[c];
        }
    }
    for (int c = 3; c >= 0; --c) {
        double s = v[c];
        for (int k = c + 1; k < 4; ++k) s -= m[c][k] * x[k];
        x[c] = s / m[c][c];
    }
    return true;
}

struct Centre {
    double t, mean, w;
};

double cost(const std::vector<Centre>& cs, const double* p) {
    double s = 0.0;
    for (const Centre& c : cs) {
        const double r = model(c.t, p) - c.mean;
        s += c.w * r * r;
    }
    return s;
}

// Levenberg-Marquardt (Marquardt's scaling by the diagonal) of the weighted
// least-squares cost, b kept above -min(t), d in [0.05, 8]
bool fit_lm(const std::vector<Centre>& cs, double* p) {
    double t_min = cs[0].t;
    for (const Centre& c : cs) t_min = std::min(t_min, c.t);
    const double b_lo = -t_min + 1e-6;
    double lambda = 1e-3, f = cost(cs, p);
    for (int it = 0; it < 2000; ++it) {
        double jtj[4][4] = {}, jtr[4] = {};
        for (const Centre& c : cs) {
            double g[4];
            grad(c.t, p, g);
            const double r = model(c.t, p) - c.mean;
            for (int i = 0; i < 4; ++i) {
                jtr[i] += c.w * g[i] * r;
                for (int k = 0; k < 4; ++k) jtj[i][k] += c.w * g[i] * g[k];
            }
        }
        bool improved = false;
        for (int tries = 0; tries < 60 && !improved; ++tries) {
            double m[4][4], v[4], dx[4] = {0, 0, 0, 0};
            for (int i = 0; i < 4; ++i) {
                for (int k = 0; k < 4; ++k) m[i][k] = jtj[i][k];
                m[i][i] += lambda * (jtj[i][i] > 0 ? jtj[i][i] : 1.0);
                v[i] = -jtr[i];
            }
            if (!solve4(m, v, dx)) {
                lambda *= 10.0;
                continue;
            }
            double q[4];
            for (int i = 0; i < 4; ++i) q[i] = p[i] + dx[i];
            if (q[1] <= b_lo || q[2] < 0.05 || q[2] > 8.0) {
                lambda *= 10.0;
                continue;
            }
            const double fq = cost(cs, q);
            if (std::isfinite(fq) && fq <= f) {
                double rel = 0.0;
                for (int i = 0; i < 4; ++i)
                    rel = std::max(rel, std::fabs(dx[i]) / std::max(std::fabs(p[i]), 1e-12));
                for (int i = 0; i < 4; ++i) p[i] = q[i];
                const double df = f - fq;
                f = fq;
                lambda = std::max(lambda * 0.1, 1e-15);
                improved = true;
                if (rel < 1e-13 || df <= 1e-16 * std::max(f, 1e-300)) return true;
            } else {
                lambda *= 10.0;
            }
        }
        if (!improved) return true;  // no step lowers the cost: a minimum
    }
    return true;
}

}  // namespace
}  // namespace tpx

using namespace tpx;

extern "C" {

size_t tpx_walk_fit_workspace_bytes(void) { return (2 * kBins + 1) * 8 + 256; }

tpx_status tpx_walk_fit(tpx_events ev, size_t n_ev, const uint64_t* trig_toa, size_t n_trig,
                        uint64_t tof_lo, uint64_t tof_hi, uint32_t min_count, double* params_h,
                        uint32_t* count_h, double* mean_h, float* lut, void* ws, size_t ws_bytes,
                        void* stream) {
    if (!params_h) return report(TPX_EINVAL, "params_h is NULL");
    if (n_ev && (!ev.tot || !ev.shot || !ev.toa || !trig_toa))
        return report(TPX_EINVAL, "an event array or trig_toa is NULL");
    if (tof_hi < tof_lo) return report(TPX_EINVAL, "tof_hi < tof_lo");
    if (min_count == 0) return report(TPX_EINVAL, "min_count must be at least 1");
    if (!ws || ws_bytes < tpx_walk_fit_workspace_bytes())
        return report(TPX_EINVAL, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* bins = (unsigned long long*)ws;
    hipLaunchKernelGGL(k_walk_clear, dim3(1), dim3(256), 0, s, bins);
    if (n_ev) {
        uint64_t blocks = (n_ev + kWalkWG - 1) / kWalkWG;
        if (blocks > kWalkBlocks) blocks = kWalkBlocks;
        hipLaunchKernelGGL(k_walk_bins, dim3((unsigned)blocks), dim3(kWalkWG), 0, s, ev,
                           (uint64_t)n_ev, trig_toa, (uint64_t)n_trig, tof_lo, tof_hi, bins);
    }
    std::vector<unsigned long long> h(2 * kBins + 1);
    if (hipMemcpyAsync(h.data(), bins, h.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return report(TPX_EHIP, "walk bins: launch or copy failed");
    }
    if (h[2 * kBins]) return report(TPX_EINVAL, "an event's shot has no trigger time");
    const double tick = 1.5625;
    std::vector<Centre> cs;
    for (int t = 0; t < kBins; ++t) {
        const double n = (double)h[t];
        const double mean = h[t] ? ((double)tof_lo + (double)h[kBins + t] / n) * tick : NAN;
        if (count_h) count_h[t] = (uint32_t)std::min<unsigned long long>(h[t], 0xFFFFFFFFull);
        if (mean_h) mean_h[t] = mean;
        if (h[t] >= min_count) cs.push_back(Centre{(double)t, mean, n});
    }
    if (cs.size() < 4) return report(TPX_EINVAL, "fewer than 4 ToT values with min_count pixels");
    // start: d = 1, b = 1, c from the brightest fifth of the ToT values, a
    // from the dimmest one
    const size_t k = std::max<size_t>(1, cs.size() / 5);
    double c0 = 0.0;
    for (size_t i = cs.size() - k; i < cs.size(); ++i) c0 += cs[i].mean;
    c0 /= (double)k;
    double p[4] = {(cs[0].mean - c0) * (cs[0].t + 1.0), 1.0, 1.0, c0};  // a, b, d, c
    if (cs[0].t + p[1] <= 0) p[1] = -cs[0].t + 1.0;
    fit_lm(cs, p);
    params_h[0] = p[0];
    params_h[1] = p[1];
    params_h[2] = p[3];
    params_h[3] = p[2];
    if (lut) {
        float tab[kBins];
        const double t_ok = std::max(0.0, std::floor(-p[1]) + 1.0);  // smallest ToT with ToT + b > 0
        for (int t = 0; t < kBins; ++t) {
            const double tt = std::max((double)t, t_ok);
            tab[t] = (float)(p[0] / std::pow(tt + p[1], p[2]));
        }
        if (hipMemcpyAsync(lut, tab, sizeof(tab), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            (void)hipGetLastError();
            return report(TPX_EHIP, "walk table copy failed");
        }
    }
    return TPX_OK;
}

}  // extern "C"
