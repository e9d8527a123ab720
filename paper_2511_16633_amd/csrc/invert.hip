// One linearised frequency set: the Hessian-free single step (paper,
// Inverse Problem section: Eqs. 8-10 and the single-step paragraph; data
// handling from the Results section).
//
//   p_er      = G_e(x_r)                    modelled data (Eq. 2, s(omega) = 1)
//   D         = p_meas - p                  residual of the objective (Eq. 8)
//   W         = receiver selection x outlier zeroing
//   grad, Hd  = J^T W D,  diag(J^T W J)     gradient and Hessian diagonal (Eq. 10)
//   v         = S grad / (Hd + eps max_S Hd)   diagonal solution-space weight
//   beta      = Re<J v, W D> / <J v, W J v>   exact minimiser along v
//   c_out     = (1/c^2 + beta v)^(-1/2)
//
// The CG variant (the paper's earlier method: the linearised equation
// H delta = J^T W D solved iteratively) shares steps 1-4 and replaces the
// single step by Jacobi-preconditioned CG on the pixels where the diagonal
// weight is defined, preconditioned by that weight, so that its first
// iterate is beta v.  Its scalars stay on the device; each iteration is one
// Born forward (p.Hp = <J p, W J p> in data space) and, except the last,
// one weighted adjoint (H p = J^T W J p).
//
// Every reduction here has a fixed order (per-block trees over a fixed grid,
// then one block), and the outlier selection uses integer keys, so the
// result does not depend on scheduling.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "born.h"
#include "common.h"
#include "green.h"

namespace rb {

size_t trace_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int batch);
rb_status trace_rays_impl(const rb_geometry *g, const rb_trace_opts *t, const double *slowness,
                          const double *alpha0, const rb_tables *out, void *ws, size_t ws_bytes, hipStream_t st,
                          uint8_t *cover, const GreenOut *gout);

namespace {

constexpr int kRB = kReduceBlocks;

__global__ void k_slowness(const double *__restrict__ c, int64_t n, double *__restrict__ s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) s[i] = 1.0 / c[i];
}

// Modelled data from the receiver tables and the residual, [nf][m][m] complex.
__global__ void k_residual(GreenParams G, int m, const double *__restrict__ Trx, const float *__restrict__ arx,
                           const float *__restrict__ brx, const double *__restrict__ pmeas,
                           double *__restrict__ D) {
    const int64_t mm = (int64_t)m * m;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= mm * G.nf) return;
    const int k = (int)(idx / mm);
    const int64_t q = idx - (int64_t)k * mm;
    const double t = Trx[q];
    double pr = 0.0, pi = 0.0;
    if (!isnan(t)) {
        const double cycles = G.f[k] * t + 0.125;
        const double frac = cycles - floor(cycles);
        double sn, cs;
        sincospi(2.0 * frac, &sn, &cs);
        const double mag = (double)arx[q] * G.rsq[k] * exp(-(double)brx[q] * G.fy[k]);
        pr = mag * cs;
        pi = mag * sn;
    }
    D[2 * idx] = pmeas[2 * idx] - pr;
    D[2 * idx + 1] = pmeas[2 * idx + 1] - pi;
}

// Receiver selection of pair (e, r): circular distance at least dmin.
__device__ __forceinline__ bool selected_er(int e, int r, int m, int dmin) {
    int d = e > r ? e - r : r - e;
    d = d < m - d ? d : m - d;
    return d >= dmin;
}

// Data weights: receiver selection, then the kzero selected pairs with the
// largest |p_meas|^2 of a frequency are zeroed (ties to the smaller flat
// index).  The kzero-th largest is found by a radix select on the IEEE bits
// of |p|^2 (non-negative doubles order like their bit patterns), stored as
// key = bits + 1 for a selected pair and 0 for the others, so the passes
// need no selection test and key 0 never reaches the threshold.  Digits are
// the 12 sign/exponent bits, then 13 mantissa bits at a time (five passes).
// The keys are parked in W, which receives the weights at the end.
//
// A frequency's m^2 flat indices are split into contiguous block ranges
// (thread t owns indices lo + t, lo + t + T, ... of its block's range, so
// every access is coalesced), and the steps are launches over all blocks of
// all frequencies:
//   k_wkeys   keys, and the histogram of the first digit;
//   k_wsel    (one block per frequency) the digit at which the count of
//             larger keys reaches the number still to zero, appended to the
//             threshold's prefix;
//   k_whist   the next digit's histogram among keys with that prefix;
//   k_wties   keys equal to the threshold, per block;
//   k_wfinal  the weights (ties ranked in flat-index order across blocks
//             only when the threshold splits them), and per block the
//             number of zeroed selected pairs;
//   k_zlist   the zeroed selected pairs as (e, r) in flat-index order, for
//             the banded Hessian diagonal.
// Histograms are integer counts (their atomics commute), so the result does
// not depend on scheduling.  A wave whose active lanes share a digit adds
// them with one LDS atomic.
constexpr int kWT = 256;            // threads per block
constexpr int kWBins = 1 << 13;     // digit bins (the first digit uses 4096)
constexpr int kWMaxBlocks = 64;     // blocks per frequency
constexpr int kWU = 4;              // stripes loaded together

// Blocks per frequency: about 32 stripes each, at most kWMaxBlocks.
inline int w_blocks(int64_t mm) {
    return (int)std::min<int64_t>(kWMaxBlocks, std::max<int64_t>(1, (mm + 32 * kWT - 1) / (32 * kWT)));
}

// The flat range [lo, hi) of block b of nb (a multiple of kWT long) and its
// number of stripes of kWT indices.
struct WRange {
    int64_t lo, hi, ns;
};
__device__ __forceinline__ WRange w_range(int64_t mm, int nb, int b) {
    const int64_t span = ((mm + nb - 1) / nb + kWT - 1) / kWT * kWT;
    WRange r;
    r.lo = min(mm, (int64_t)b * span);
    r.hi = min(mm, r.lo + span);
    r.ns = (r.hi - r.lo + kWT - 1) / kWT;
    return r;
}

// Exclusive prefix sum of v over the kWT threads of the block in thread
// order (wave scans by shuffles, then the wave totals); `total` receives the
// block sum.  Every thread of the block must call it.
__device__ __forceinline__ int64_t w_exscan(int64_t v, int64_t *s_w, int64_t &total) {
    constexpr int NW = kWT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const int64_t t = s_w[q];
        if (q < w) base += t;
        tot += t;
    }
    total = tot;
    __syncthreads();   // s_w may be reused
    return base + x - v;
}

// Adds digit dg of the lanes with `on` to an LDS histogram.  Every lane of
// the wave calls it.
__device__ __forceinline__ void w_hist_add(unsigned *hist, bool on, unsigned dg) {
    const uint64_t act = __ballot(on);
    if (act == 0) return;   // wave-uniform
    const int first = __ffsll((unsigned long long)act) - 1;
    const unsigned d0 = __shfl(dg, first);
    if (__ballot(on && dg != d0) == 0) {
        if ((int)(threadIdx.x & 63) == first) atomicAdd(&hist[d0], (unsigned)__popcll(act));
    } else if (on) {
        atomicAdd(&hist[dg], 1u);
    }
}

// Adds the block's LDS histogram to the frequency's global one.
__device__ __forceinline__ void w_hist_flush(const unsigned *hist, int nbins, unsigned *gh) {
    __syncthreads();
    for (int q = threadIdx.x; q < nbins; q += kWT) {
        const unsigned c = hist[q];
        if (c) atomicAdd(&gh[q], c);
    }
}

// Keys (or, with kzero <= 0, the selection weights themselves) and the
// first digit's histogram.  Grid (nb, nf).
__global__ void __launch_bounds__(kWT) k_wkeys(int m, int dmin, int nb, int64_t kzero,
                                               const double *__restrict__ pmeas, double *__restrict__ W,
                                               unsigned *__restrict__ whist) {
    __shared__ unsigned hist[1 << 12];
    const int b = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
    const int64_t mm = (int64_t)m * m;
    const WRange R = w_range(mm, nb, b);
    const double *pk = pmeas + 2 * (int64_t)k * mm;
    double *wk = W + (int64_t)k * mm;
    uint64_t *keys = reinterpret_cast<uint64_t *>(wk);
    const bool sel_only = kzero <= 0;   // kernel-uniform
    if (!sel_only) {
        for (int q = t; q < (1 << 12); q += kWT) hist[q] = 0;
        __syncthreads();
    }
    for (int64_t s0 = 0; s0 < R.ns; s0 += kWU) {
        double re[kWU], im[kWU];
        bool sel[kWU];
#pragma unroll
        for (int u = 0; u < kWU; ++u) {
            const int64_t i = R.lo + (s0 + u) * kWT + t;
            const bool ok = s0 + u < R.ns && i < R.hi;
            const int e = ok ? (int)(i / m) : 0, r = ok ? (int)(i - (int64_t)e * m) : 0;
            sel[u] = ok && selected_er(e, r, m, dmin);
            re[u] = (sel[u] && !sel_only) ? pk[2 * i] : 0.0;
            im[u] = (sel[u] && !sel_only) ? pk[2 * i + 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kWU; ++u) {
            const int64_t i = R.lo + (s0 + u) * kWT + t;
            const bool ok = s0 + u < R.ns && i < R.hi;
            if (sel_only) {
                if (ok) wk[i] = sel[u] ? 1.0 : 0.0;
                continue;
            }
            const uint64_t key =
                sel[u] ? (uint64_t)__double_as_longlong(re[u] * re[u] + im[u] * im[u]) + 1ull : 0ull;
            if (ok) keys[i] = key;
            w_hist_add(hist, key != 0, (unsigned)(key >> 52));
        }
    }
    if (sel_only) return;
    w_hist_flush(hist, 1 << 12, whist + (int64_t)k * kWBins);
}

// Digit `pass` of the threshold (one block per frequency): the largest digit
// value at which the count of keys with larger digits (and the prefix so
// far) reaches the number still to zero.  State per frequency: the
// threshold's prefix and that number.  Clears the histogram for the next
// pass once every thread has read its bins.
__global__ void __launch_bounds__(kWT) k_wsel(int pass, int64_t kzero, unsigned *__restrict__ whist,
                                              uint64_t *__restrict__ wstate) {
    __shared__ int64_t s_w[kWT / 64];
    constexpr int D = kWBins / kWT;
    const int k = blockIdx.x, t = threadIdx.x;
    const int width = pass == 0 ? 12 : 13;
    const int shift = 52 - 13 * pass;   // 52, 39, 26, 13, 0
    const int nbins = 1 << width, dpt = nbins / kWT;
    unsigned *gh = whist + (int64_t)k * kWBins;
    const uint64_t pref = pass == 0 ? 0ull : wstate[2 * k];
    const int64_t rem = pass == 0 ? kzero : (int64_t)wstate[2 * k + 1];
    if (pass == 0 && t == 0) {   // ordered before the choice below by the scan's barriers
        wstate[2 * k] = 0ull;
        wstate[2 * k + 1] = (uint64_t)kzero;
    }
    // thread t holds the digits nbins - 1 - (dpt t + u), u < dpt (descending)
    unsigned c[D];
    int64_t cnt = 0;
#pragma unroll
    for (int u = 0; u < D; ++u) {
        c[u] = u < dpt ? gh[nbins - 1 - (dpt * t + u)] : 0u;
        cnt += c[u];
    }
    int64_t tot;
    int64_t ex = w_exscan(cnt, s_w, tot);
    if (cnt > 0 && ex < rem && ex + cnt >= rem) {
        for (int u = 0; u < dpt; ++u) {
            if (c[u] > 0 && ex + (int64_t)c[u] >= rem) {
                wstate[2 * k] = pref | ((uint64_t)(nbins - 1 - (dpt * t + u)) << shift);
                wstate[2 * k + 1] = (uint64_t)(rem - ex);
                break;
            }
            ex += c[u];
        }
    }
    for (int q = t; q < kWBins; q += kWT) gh[q] = 0;
}

// Histogram of digit `pass` (1..4) among the keys that carry the threshold's
// prefix.  Grid (nb, nf).
__global__ void __launch_bounds__(kWT) k_whist(int pass, int m, int nb, const double *__restrict__ W,
                                               const uint64_t *__restrict__ wstate, unsigned *__restrict__ whist) {
    __shared__ unsigned hist[kWBins];
    const int b = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
    const int64_t mm = (int64_t)m * m;
    const WRange R = w_range(mm, nb, b);
    const uint64_t *keys = reinterpret_cast<const uint64_t *>(W + (int64_t)k * mm);
    for (int q = t; q < kWBins; q += kWT) hist[q] = 0;
    __syncthreads();
    const int shift = 52 - 13 * pass;
    const uint64_t hmask = ~0ull << (shift + 13);
    const uint64_t pref = wstate[2 * k] & hmask;
    for (int64_t s0 = 0; s0 < R.ns; s0 += kWU) {
        uint64_t kv[kWU];
#pragma unroll
        for (int u = 0; u < kWU; ++u) {
            const int64_t i = R.lo + (s0 + u) * kWT + t;
            kv[u] = (s0 + u < R.ns && i < R.hi) ? keys[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kWU; ++u)
            w_hist_add(hist, kv[u] != 0 && (kv[u] & hmask) == pref, (unsigned)(kv[u] >> shift) & (kWBins - 1u));
    }
    w_hist_flush(hist, kWBins, whist + (int64_t)k * kWBins);
}

// Keys equal to the threshold, per block.  Grid (nb, nf).
__global__ void __launch_bounds__(kWT) k_wties(int m, int nb, const double *__restrict__ W,
                                               const uint64_t *__restrict__ wstate, int64_t *__restrict__ wcnt) {
    __shared__ int64_t s_w[kWT / 64];
    const int b = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
    const int64_t mm = (int64_t)m * m;
    const WRange R = w_range(mm, nb, b);
    const uint64_t *keys = reinterpret_cast<const uint64_t *>(W + (int64_t)k * mm);
    const uint64_t kstar = wstate[2 * k];
    int64_t n = 0;
    for (int64_t s = 0; s < R.ns; ++s) {
        const int64_t i = R.lo + s * kWT + t;
        if (i < R.hi && keys[i] == kstar) ++n;
    }
    int64_t tot;
    (void)w_exscan(n, s_w, tot);
    if (t == 0) wcnt[(int64_t)k * kWMaxBlocks + b] = tot;
}

// The weights in place of the keys; per block, the number of zeroed
// selected pairs.  Grid (nb, nf).
__global__ void __launch_bounds__(kWT) k_wfinal(int m, int nb, double *__restrict__ W,
                                                const uint64_t *__restrict__ wstate, const int64_t *__restrict__ wcnt,
                                                int64_t *__restrict__ zcnt) {
    __shared__ int64_t s_w[kWT / 64];
    const int b = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
    const int64_t mm = (int64_t)m * m;
    const WRange R = w_range(mm, nb, b);
    double *wk = W + (int64_t)k * mm;
    const uint64_t *keys = reinterpret_cast<const uint64_t *>(wk);
    const uint64_t kstar = wstate[2 * k];          // a selected key (>= 1)
    const int64_t need = (int64_t)wstate[2 * k + 1];   // keys equal to kstar to zero, lowest flat index first
    int64_t nties = 0, base = 0;   // all ties; ties in earlier blocks
    for (int q = 0; q < nb; ++q) {
        const int64_t c = wcnt[(int64_t)k * kWMaxBlocks + q];
        nties += c;
        if (q < b) base += c;
    }
    // all ties zeroed (need == nties) or none (need == 0) needs no ranks
    const bool ranked = need > 0 && need < nties;   // kernel-uniform
    int64_t zc = 0;
    for (int64_t s = 0; s < R.ns; ++s) {
        const int64_t i = R.lo + s * kWT + t;
        const bool ok = i < R.hi;
        const uint64_t key = ok ? keys[i] : 0ull;
        double w = (key == 0 || key > kstar) ? 0.0 : 1.0;
        const bool tie = key == kstar;
        if (tie && !ranked && need > 0) w = 0.0;
        if (ranked) {
            int64_t st;
            const int64_t ex = w_exscan(tie ? 1 : 0, s_w, st);
            if (tie && base + ex < need) w = 0.0;
            base += st;
        }
        if (ok) {
            wk[i] = w;   // replaces this thread's own key
            if (key != 0 && w == 0.0) ++zc;
        }
    }
    int64_t tot;
    (void)w_exscan(zc, s_w, tot);
    if (t == 0) zcnt[(int64_t)k * kWMaxBlocks + b] = tot;
}

// The zeroed selected pairs of each frequency as (e, r) in flat-index order,
// at most zcap of them, and their count.  Grid (nb, nf).
__global__ void __launch_bounds__(kWT) k_zlist(int m, int dmin, int nb, const double *__restrict__ W,
                                               const int64_t *__restrict__ zcnt, int zcap, int2 *__restrict__ zl,
                                               int *__restrict__ nz) {
    __shared__ int64_t s_w[kWT / 64];
    const int b = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
    const int64_t mm = (int64_t)m * m;
    const WRange R = w_range(mm, nb, b);
    const double *wk = W + (int64_t)k * mm;
    int64_t total = 0, pos = 0;   // all zeroed pairs; those in earlier blocks
    for (int q = 0; q < nb; ++q) {
        const int64_t c = zcnt[(int64_t)k * kWMaxBlocks + q];
        total += c;
        if (q < b) pos += c;
    }
    if (b == 0 && t == 0) nz[k] = (int)min(total, (int64_t)zcap);
    for (int64_t s = 0; s < R.ns && pos < zcap; ++s) {   // block-uniform
        const int64_t i = R.lo + s * kWT + t;
        const bool ok = i < R.hi;
        const int e = ok ? (int)(i / m) : 0, r = ok ? (int)(i - (int64_t)e * m) : 0;
        const bool z = ok && selected_er(e, r, m, dmin) && wk[i] == 0.0;
        int64_t st;
        const int64_t ex = w_exscan(z ? 1 : 0, s_w, st);
        if (z && pos + ex < zcap) zl[(int64_t)k * zcap + pos + ex] = make_int2(e, r);
        pos += st;
    }
}

// Support, part 1: |x| < R - margin.  The rasteriser's write pass then
// clears every pixel that some emitter does not cover.
__global__ void k_support_disc(int nx, int ny, double h, double x0, double y0, double rs,
                               uint8_t *__restrict__ S) {
    const int64_t N = (int64_t)nx * ny;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t j = p / nx, i = p - j * nx;
    const double px = x0 + (double)i * h, py = y0 + (double)j * h;
    S[p] = (px * px + py * py < rs * rs) ? 1 : 0;
}

__global__ void k_direction(int64_t n, const double *__restrict__ grad, const double *__restrict__ hd,
                            const uint8_t *__restrict__ S, const double *__restrict__ hmax, double eps,
                            double *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double hm = hmax[0] > -INFINITY ? hmax[0] : 0.0;
    const double den = hd[i] + eps * hm;
    v[i] = (S[i] && den > 0.0) ? grad[i] / den : 0.0;
}

// Fixed-order block sums: partial[b][0..1] over a fixed strided index set.
__global__ void k_beta_partial(int64_t n, const double *__restrict__ W, const double *__restrict__ u,
                               const double *__restrict__ D, double *__restrict__ part) {
    __shared__ double sn[256], sd[256];
    double num = 0.0, den = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double w = W[i];
        const double ur = u[2 * i], ui = u[2 * i + 1];
        num += w * (ur * D[2 * i] + ui * D[2 * i + 1]);
        den += w * (ur * ur + ui * ui);
    }
    sn[threadIdx.x] = num;
    sd[threadIdx.x] = den;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sn[threadIdx.x] += sn[threadIdx.x + s];
            sd[threadIdx.x] += sd[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sn[0];
        part[2 * blockIdx.x + 1] = sd[0];
    }
}

// res[0] = num, res[1] = den, res[2] = beta
__global__ void k_beta_final(const double *__restrict__ part, int np, double *__restrict__ res) {
    __shared__ double sn[256], sd[256];
    double num = 0.0, den = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) {
        num += part[2 * i];
        den += part[2 * i + 1];
    }
    sn[threadIdx.x] = num;
    sd[threadIdx.x] = den;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sn[threadIdx.x] += sn[threadIdx.x + s];
            sd[threadIdx.x] += sd[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        res[0] = sn[0];
        res[1] = sd[0];
        res[2] = sd[0] > 0.0 ? sn[0] / sd[0] : 0.0;
    }
}

// Update check: sum of (c_new - c)^2 and count of non-positive q.
__global__ void k_update_partial(int64_t n, const double *__restrict__ c, const double *__restrict__ s,
                                 const double *__restrict__ v, const double *__restrict__ res,
                                 double *__restrict__ part) {
    __shared__ double ss[256], sb[256];
    const double beta = res[2];
    double sq = 0.0, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double delta = beta * v[i];
        if (delta != 0.0) {
            const double q = s[i] * s[i] + delta;
            if (q <= 0.0) {
                bad += 1.0;
            } else {
                const double dc = 1.0 / sqrt(q) - c[i];
                sq += dc * dc;
            }
        }
    }
    ss[threadIdx.x] = sq;
    sb[threadIdx.x] = bad;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            ss[threadIdx.x] += ss[threadIdx.x + st];
            sb[threadIdx.x] += sb[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss[0];
        part[2 * blockIdx.x + 1] = sb[0];
    }
}

// res[3] = sum dc^2, res[4] = number of non-positive q
__global__ void k_update_final(const double *__restrict__ part, int np, double *__restrict__ res) {
    __shared__ double ss[256], sb[256];
    double sq = 0.0, bad = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) {
        sq += part[2 * i];
        bad += part[2 * i + 1];
    }
    ss[threadIdx.x] = sq;
    sb[threadIdx.x] = bad;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            ss[threadIdx.x] += ss[threadIdx.x + st];
            sb[threadIdx.x] += sb[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        res[3] = ss[0];
        res[4] = sb[0];
    }
}

__global__ void k_update_write(int64_t n, const double *c, const double *__restrict__ s,
                               const double *__restrict__ v, const double *__restrict__ res, double *c_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ci = c[i];
    double out = ci;
    if (res[4] == 0.0) {
        const double delta = res[2] * v[i];
        if (delta != 0.0) out = 1.0 / sqrt(s[i] * s[i] + delta);
    }
    c_out[i] = out;
}

// ------------------------------------------------------------------ CG
// Device state cg[]: 0 r.z, 1 alpha, 2 beta, 3 stopped (nonzero once r.z or
// p.Hp has not been positive; every later step is then zero).  hist[2 i] is
// iteration i's alpha, hist[2 i + 1] its r.z (both 0 for iterations after a
// stop).

__device__ __forceinline__ bool cg_ok(const uint8_t *S, const double *hd, int64_t i, double eps_hm, double &den) {
    den = hd[i] + eps_hm;
    return S[i] && den > 0.0;
}

// Block tree of one value per thread into part[blockIdx.x].
__device__ __forceinline__ void block_sum_to(double v, double *s_red, double *part) {
    s_red[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) s_red[threadIdx.x] += s_red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s_red[0];
}

// x = 0, r = grad on ok (0 elsewhere), z = p = r / den (the single step's v);
// partial sums of r.z.
__global__ void k_cg_start(int64_t n, const double *__restrict__ grad, const double *__restrict__ hd,
                           const uint8_t *__restrict__ S, const double *__restrict__ hmax, double eps,
                           double *__restrict__ x, double *__restrict__ r, double *__restrict__ z,
                           double *__restrict__ p, double *__restrict__ part) {
    __shared__ double s_red[256];
    const double hm = hmax[0] > -INFINITY ? hmax[0] : 0.0;
    const double eps_hm = eps * hm;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double den;
        const bool ok = cg_ok(S, hd, i, eps_hm, den);
        const double ri = ok ? grad[i] : 0.0;
        const double zi = ok ? grad[i] / den : 0.0;
        x[i] = 0.0;
        r[i] = ri;
        z[i] = zi;
        p[i] = zi;
        acc += ri * zi;
    }
    block_sum_to(acc, s_red, part);
}

// Sum of the r.z partials.  first: cg[0] = r.z, nothing stopped.  Else
// beta = new / old (0 once stopped) and cg[0] = new.
__global__ void k_cg_rz_final(const double *__restrict__ part, int np, double *__restrict__ cg, int first) {
    __shared__ double s_red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
    s_red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) s_red[threadIdx.x] += s_red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double rz = s_red[0];
        if (first) {
            cg[3] = 0.0;
        } else {
            cg[2] = (cg[3] == 0.0 && cg[0] > 0.0) ? rz / cg[0] : 0.0;
        }
        cg[0] = rz;
    }
}

// alpha = r.z / p.Hp from the partials of <J p, W J p> (second component of
// the step-length partials); stop on a non-positive r.z or p.Hp.
__global__ void k_cg_alpha(const double *__restrict__ part, int np, double *__restrict__ cg,
                           double *__restrict__ hist, int it) {
    __shared__ double s_red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) acc += part[2 * i + 1];
    s_red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) s_red[threadIdx.x] += s_red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double a = 0.0, rz = 0.0;
        if (cg[3] == 0.0) {
            rz = cg[0];
            const double pq = s_red[0];
            if (rz > 0.0 && pq > 0.0)
                a = rz / pq;
            else
                cg[3] = 1.0;
        }
        cg[1] = a;
        hist[2 * it] = a;
        hist[2 * it + 1] = rz;
    }
}

// x += alpha p; r -= alpha q on ok; z = r / den on ok; partial sums of r.z.
__global__ void k_cg_step(int64_t n, const double *__restrict__ q, const double *__restrict__ hd,
                          const uint8_t *__restrict__ S, const double *__restrict__ hmax, double eps,
                          const double *__restrict__ cg, double *__restrict__ x, const double *__restrict__ p,
                          double *__restrict__ r, double *__restrict__ z, double *__restrict__ part) {
    __shared__ double s_red[256];
    const double hm = hmax[0] > -INFINITY ? hmax[0] : 0.0;
    const double eps_hm = eps * hm;
    const double a = cg[1];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double den;
        const bool ok = cg_ok(S, hd, i, eps_hm, den);
        x[i] = x[i] + a * p[i];
        const double ri = ok ? r[i] - a * q[i] : r[i];
        const double zi = ok ? ri / den : 0.0;
        r[i] = ri;
        z[i] = zi;
        acc += ri * zi;
    }
    block_sum_to(acc, s_red, part);
}

// p = z + beta p
__global__ void k_cg_direction(int64_t n, const double *__restrict__ z, const double *__restrict__ cg,
                               double *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + cg[2] * p[i];
}

// x += alpha p (last iteration); res[2] = 1 so that the update kernels
// apply delta = x.
__global__ void k_cg_last(int64_t n, const double *__restrict__ cg, const double *__restrict__ p,
                          double *__restrict__ x, double *__restrict__ res) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = x[i] + cg[1] * p[i];
    if (i == 0) res[2] = 1.0;
}

// ------------------------------------------------------ asymptotic weights
// Tables for the amplitude-normalised backprojection: H = G / |G|^2 (so
// conj(H_e H_r) = 1 / (G_e G_r)) and the coverage indicator C = [G != 0].
template <typename T>
__global__ void k_asym_tables(int64_t n, const T *__restrict__ Gr, const T *__restrict__ Gi, T *__restrict__ Hr,
                              T *__restrict__ Hi, T *__restrict__ C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T a = Gr[i], b = Gi[i];
    const T h = a * a + b * b;
    const bool nz = a != T(0) || b != T(0);
    Hr[i] = nz ? a / h : T(0);
    Hi[i] = nz ? b / h : T(0);
    C[i] = nz ? T(1) : T(0);
}

// gA += sg gk, nA += sn nk
__global__ void k_asym_accum(int64_t n, const double *__restrict__ gk, const double *__restrict__ nk, double sg,
                             double sn, double *__restrict__ gA, double *__restrict__ nA) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    gA[i] += sg * gk[i];
    nA[i] += sn * nk[i];
}

__global__ void k_asym_direction(int64_t n, const double *__restrict__ gA, const double *__restrict__ nA,
                                 const uint8_t *__restrict__ S, double *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    v[i] = (S[i] && nA[i] > 0.0) ? gA[i] / nA[i] : 0.0;
}

struct InvWs {
    double *s, *T, *Trx, *D, *W, *Jv, *grad, *hd, *v, *part, *res, *hmax;
    float *amp, *att, *amp_rx, *att_rx, *gscale;
    void *Gr, *Gi;
    uint8_t *S;
    int2 *zl;   // zeroed pairs [nf][m m]
    int *nz;    // their counts [nf]
    unsigned *whist;        // outlier selection: digit histograms [nf][kWBins]
    uint64_t *wstate;       // threshold prefix and count still to zero [nf][2]
    int64_t *wcnt, *zcnt;   // per-block ties and zeroed pairs [nf][kWMaxBlocks]
    double *x, *r, *z, *p, *q, *cg, *hist;   // CG only
    void *Hr, *Hi, *C, *C0;                   // asymptotic weights only
    double *gk, *nk, *gA, *nA;
    void *scratch;
};

InvWs carve_inv(Carver &c, const rb_geometry *g, int nf, rb_dtype dt, bool cg, bool asym = false) {
    const size_t N = (size_t)g->nx * g->ny, m = g->m, mm = m * m;
    const size_t es = dtype_size(dt);
    InvWs w;
    w.s = c.take<double>(N);
    w.T = c.take<double>(m * N);
    w.amp = c.take<float>(m * N);
    w.att = c.take<float>(m * N);
    w.Trx = c.take<double>(mm);
    w.amp_rx = c.take<float>(mm);
    w.att_rx = c.take<float>(mm);
    w.Gr = c.take<char>((size_t)nf * m * N * es);
    w.Gi = c.take<char>((size_t)nf * m * N * es);
    w.gscale = c.take<float>(RB_MAX_NF);
    w.D = c.take<double>((size_t)nf * mm * 2);
    w.W = c.take<double>((size_t)nf * mm);
    w.Jv = c.take<double>((size_t)nf * mm * 2);
    w.grad = c.take<double>(N);
    w.hd = c.take<double>(N);
    w.v = c.take<double>(N);
    w.S = c.take<uint8_t>(N);
    w.part = c.take<double>(2 * kRB);
    w.res = c.take<double>(8);
    w.hmax = c.take<double>(1);
    w.zl = c.take<int2>((size_t)nf * mm);
    w.nz = c.take<int>(RB_MAX_NF);
    w.whist = c.take<unsigned>((size_t)nf * kWBins);
    w.wstate = c.take<uint64_t>((size_t)2 * nf);
    w.wcnt = c.take<int64_t>((size_t)nf * kWMaxBlocks);
    w.zcnt = c.take<int64_t>((size_t)nf * kWMaxBlocks);
    w.x = w.r = w.z = w.p = w.q = w.cg = w.hist = nullptr;
    if (cg) {
        w.x = c.take<double>(N);
        w.r = c.take<double>(N);
        w.z = c.take<double>(N);
        w.p = c.take<double>(N);
        w.q = c.take<double>(N);
        w.cg = c.take<double>(8);
        w.hist = c.take<double>(2 * RB_MAX_CG_ITERS);
    }
    w.Hr = w.Hi = w.C = w.C0 = nullptr;
    w.gk = w.nk = w.gA = w.nA = nullptr;
    if (asym) {
        w.Hr = c.take<char>((size_t)nf * m * N * es);
        w.Hi = c.take<char>((size_t)nf * m * N * es);
        w.C = c.take<char>((size_t)nf * m * N * es);
        w.C0 = c.take<char>((size_t)m * N * es);
        w.gk = c.take<double>(N);
        w.nk = c.take<double>(N);
        w.gA = c.take<double>(N);
        w.nA = c.take<double>(N);
    }
    w.scratch = c.take<char>(0);
    return w;
}

size_t scratch_need(const rb_geometry *g, const rb_trace_opts *t, int nf, rb_dtype dt, int batch) {
    size_t s = trace_workspace_bytes(g, t, batch);
    s = std::max(s, adjoint_workspace_bytes(g, nf, dt));
    s = std::max(s, forward_workspace_bytes(g, nf, dt));
    s = std::max(s, green_workspace_bytes());
    return s;
}

int selected_count(int m, int dmin) {
    int n = 0;
    for (int r = 0; r < m; ++r) {
        int d = std::min(r, m - r);
        if (d >= dmin) ++n;
    }
    return n;
}

}  // namespace

size_t invert_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int nf, rb_dtype dt, int batch,
                              bool cg, bool asym = false) {
    Carver c(nullptr, 0);
    carve_inv(c, g, nf, dt, cg, asym);
    return c.used + 256 + scratch_need(g, t, nf, dt, batch);
}

// Everything one call on one frequency set carries between its phases.
struct SetCtx {
    const rb_geometry *g;
    const rb_trace_opts *t;
    const rb_invert_opts *o;
    const double *c_in, *alpha0, *freqs, *p_meas;
    int nf;
    double *c_out;
    InvWs w;
    void *scratch;
    size_t scratch_bytes;
    int dmin;
    AdjTask adj;      // the single step's backprojection, prepared
    double res[8];    // host copy of the set's scalars
};

// Workspace carve and size check.
static rb_status set_open(SetCtx &S, const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o,
                          const double *c_in, const double *alpha0, const double *freqs, int nf,
                          const double *p_meas, double *c_out, void *ws, size_t ws_bytes, bool cg, bool asym) {
    S.g = g;
    S.t = t;
    S.o = o;
    S.c_in = c_in;
    S.alpha0 = alpha0;
    S.freqs = freqs;
    S.nf = nf;
    S.p_meas = p_meas;
    S.c_out = c_out;
    Carver c(ws, ws_bytes);
    S.w = carve_inv(c, g, nf, o->dtype, cg, asym);
    if (c.used + 256 + trace_workspace_bytes(g, t, 1) > ws_bytes ||
        c.used + 256 + std::max(adjoint_workspace_bytes(g, nf, o->dtype),
                                forward_workspace_bytes(g, nf, o->dtype)) > ws_bytes) {
        set_error("invert workspace too small (%zu bytes)", ws_bytes);
        return RB_ENOMEM;
    }
    S.scratch_bytes = ws_bytes - c.used - 256;
    S.scratch = reinterpret_cast<void *>(((uintptr_t)S.w.scratch + 255) & ~(uintptr_t)255);
    S.dmin = (int)std::ceil((1.0 - o->recv_fraction) * 0.5 * g->m - 1e-9);
    return RB_OK;
}

// 1-2. rays, tables and Green's functions in the current model; residual,
// data weights and the list of zeroed pairs
// scale[k] = omega_k^-1/2: the per-frequency scale of BF16 Green's tables
// written as G / omega^-1/2
__global__ void k_rsq_scales(GreenParams P, float *__restrict__ scale) {
    const int k = threadIdx.x;
    if (k < P.nf) scale[k] = (float)P.rsq[k];
}

static rb_status set_linearise(SetCtx &S, hipStream_t st) {
    const rb_geometry *g = S.g;
    const rb_invert_opts *o = S.o;
    InvWs &w = S.w;
    const int64_t N = (int64_t)g->nx * g->ny;
    const int m = g->m, nf = S.nf;
    const int64_t mm = (int64_t)m * m;
    k_slowness<<<blocks_for(N, 256), 256, 0, st>>>(S.c_in, N, w.s);
    RB_LAUNCHED();
    // support (step 4): inside the ring margin and covered by every emitter
    const double rs = g->ring_radius - g->support_margin;
    k_support_disc<<<blocks_for(N, 256), 256, 0, st>>>(g->nx, g->ny, g->h, g->x0, g->y0, rs, w.S);
    RB_LAUNCHED();
    rb_tables tab{w.T, w.amp, w.att, w.Trx, w.amp_rx, w.att_rx};
    if (o->dtype != RB_F16) {
        // 32/64-bit and BF16 G need no global scale: the rasteriser writes it
        // directly (BF16 as G / omega^-1/2, whose range BF16 holds); FP16,
        // with its 5-bit exponent, is normalised by the largest amplitude
        // in a pass of its own
        const GreenParams GP = green_params(S.freqs, nf, o->y_pow);
        GreenOut gout{GP, o->dtype, w.Gr, w.Gi};
        RB_TRY(trace_rays_impl(g, S.t, w.s, S.alpha0, &tab, S.scratch, S.scratch_bytes, st, w.S, &gout));
        if (o->dtype == RB_BF16) {
            k_rsq_scales<<<1, RB_MAX_NF, 0, st>>>(GP, w.gscale);
            RB_LAUNCHED();
        } else {
            RB_TRY(fill_f32(w.gscale, 1.0f, nf, st));
        }
    } else {
        RB_TRY(trace_rays_impl(g, S.t, w.s, S.alpha0, &tab, S.scratch, S.scratch_bytes, st, w.S, nullptr));
        Carver gc(S.scratch, S.scratch_bytes);
        float *amax = gc.take<float>(1);
        float *parts = gc.take<float>(kReduceBlocks);
        RB_TRY(build_green_impl(w.T, w.amp, w.att, (int64_t)m * N, S.freqs, nf, o->y_pow, o->dtype, w.Gr, w.Gi,
                                w.gscale, amax, parts, st));
    }
    GreenParams GP = green_params(S.freqs, nf, o->y_pow);
    k_residual<<<blocks_for(mm * nf, 256), 256, 0, st>>>(GP, m, w.Trx, w.amp_rx, w.att_rx, S.p_meas, w.D);
    RB_LAUNCHED();
    const int64_t n_valid = (int64_t)m * selected_count(m, S.dmin);
    const int64_t kzero = (int64_t)std::floor(o->outlier_fraction * (double)n_valid);
    const int nbw = w_blocks(mm);
    const dim3 gw(nbw, nf);
    if (kzero <= 0) {   // selection only: no pair is zeroed
        k_wkeys<<<gw, kWT, 0, st>>>(m, S.dmin, nbw, kzero, S.p_meas, w.W, w.whist);
        RB_LAUNCHED();
        return fill_f32(reinterpret_cast<float *>(w.nz), 0.0f, nf, st);   // zero bits: count 0
    }
    RB_TRY(fill_u64(reinterpret_cast<uint64_t *>(w.whist), 0ull, (int64_t)nf * kWBins / 2, st));
    k_wkeys<<<gw, kWT, 0, st>>>(m, S.dmin, nbw, kzero, S.p_meas, w.W, w.whist);
    RB_LAUNCHED();
    for (int pass = 0; pass < 5; ++pass) {
        k_wsel<<<nf, kWT, 0, st>>>(pass, kzero, w.whist, w.wstate);
        RB_LAUNCHED();
        if (pass < 4) {
            k_whist<<<gw, kWT, 0, st>>>(pass + 1, m, nbw, w.W, w.wstate, w.whist);
            RB_LAUNCHED();
        }
    }
    k_wties<<<gw, kWT, 0, st>>>(m, nbw, w.W, w.wstate, w.wcnt);
    RB_LAUNCHED();
    k_wfinal<<<gw, kWT, 0, st>>>(m, nbw, w.W, w.wstate, w.wcnt, w.zcnt);
    RB_LAUNCHED();
    // the Hessian diagonal comes from the band structure of W: the
    // backprojection computes the gradient only
    k_zlist<<<gw, kWT, 0, st>>>(m, S.dmin, nbw, w.W, w.zcnt, m * m, w.zl, w.nz);
    RB_LAUNCHED();
    return RB_OK;
}

// 6. update of 1/c^2 along res[2] * dir and the update norm; the set's
// scalars are copied to S.res (the caller synchronises the stream)
static rb_status set_update(SetCtx &S, const double *dir, hipStream_t st) {
    const int64_t N = (int64_t)S.g->nx * S.g->ny;
    InvWs &w = S.w;
    k_update_partial<<<kRB, 256, 0, st>>>(N, S.c_in, w.s, dir, w.res, w.part);
    RB_LAUNCHED();
    k_update_final<<<1, 256, 0, st>>>(w.part, kRB, w.res);
    RB_LAUNCHED();
    k_update_write<<<blocks_for(N, 256), 256, 0, st>>>(N, S.c_in, w.s, dir, w.res, S.c_out);
    RB_LAUNCHED();
    RB_HIP(hipMemcpyAsync(S.res, w.res, sizeof(S.res), hipMemcpyDeviceToHost, st));
    return RB_OK;
}

// After the stream has been synchronised: the update norm, or RB_ENUMERIC.
static rb_status set_result(const SetCtx &S, double *dc_l2) {
    if (S.res[4] != 0.0) {
        if (dc_l2) *dc_l2 = 0.0;
        set_error("1/c^2 + delta <= 0 at %.0f pixels; model left unchanged", S.res[4]);
        return RB_ENUMERIC;
    }
    if (dc_l2) *dc_l2 = std::sqrt(S.res[3]);
    return RB_OK;
}

// The single step before the backprojection's contraction: linearisation,
// cleared gradient and Hessian diagonal, the backprojection's operands.
static rb_status step_begin(SetCtx &S, hipStream_t st) {
    RB_TRY(set_linearise(S, st));
    const int64_t N = (int64_t)S.g->nx * S.g->ny;
    InvWs &w = S.w;
    RB_TRY(fill_f64(w.grad, 0.0, N, st));
    RB_TRY(fill_f64(w.hd, 0.0, N, st));
    return adjoint_prepare(S.g, w.Gr, w.Gi, w.gscale, S.o->dtype, S.freqs, S.nf, w.D, w.W, w.grad, nullptr,
                           S.scratch, S.scratch_bytes, st, &S.adj);
}

// The single step after the backprojection: Hessian diagonal, direction,
// exact step length, update.
static rb_status step_end(SetCtx &S, hipStream_t st) {
    const rb_geometry *g = S.g;
    InvWs &w = S.w;
    const int64_t N = (int64_t)g->nx * g->ny;
    const int m = g->m;
    const int64_t mm = (int64_t)m * m;
    RB_TRY(hessian_band_impl(g, w.Gr, w.Gi, w.gscale, S.o->dtype, S.freqs, S.nf, S.dmin,
                             reinterpret_cast<int *>(w.zl), w.nz, m * m, w.hd, st));
    RB_TRY(reduce_max_f64(w.hd, w.S, N, w.part, w.hmax, st));
    // 4. diagonally weighted direction on the support
    k_direction<<<blocks_for(N, 256), 256, 0, st>>>(N, w.grad, w.hd, w.S, w.hmax, S.o->eps, w.v);
    RB_LAUNCHED();
    // 5. exact step length along v
    RB_TRY(forward_impl(g, w.Gr, w.Gi, w.gscale, S.o->dtype, S.freqs, S.nf, w.v, w.Jv, S.scratch,
                        S.scratch_bytes, st, S.dmin));
    k_beta_partial<<<kRB, 256, 0, st>>>(mm * S.nf, w.W, w.Jv, w.D, w.part);
    RB_LAUNCHED();
    k_beta_final<<<1, 256, 0, st>>>(w.part, kRB, w.res);
    RB_LAUNCHED();
    return set_update(S, w.v, st);
}

// cg_iters = 0: the single step; cg_iters >= 1: CG (cg_hist [host] may be
// null); asym: the single step with the asymptotic weights (32/64-bit).
rb_status invert_impl(const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o, const double *c_in,
                      const double *alpha0, const double *freqs, int nf, const double *p_meas, int cg_iters,
                      double *c_out, double *dc_l2, double *cg_hist, void *ws, size_t ws_bytes, hipStream_t st,
                      bool asym = false) {
    SetCtx S;
    RB_TRY(set_open(S, g, t, o, c_in, alpha0, freqs, nf, p_meas, c_out, ws, ws_bytes, cg_iters > 0, asym));
    if (cg_iters == 0 && !asym) {
        RB_TRY(step_begin(S, st));
        RB_TRY(adjoint_run(S.adj, st));
        RB_TRY(step_end(S, st));
        RB_HIP(hipStreamSynchronize(st));
        return set_result(S, dc_l2);
    }
    InvWs &w = S.w;
    void *scratch = S.scratch;
    const size_t scratch_bytes = S.scratch_bytes;
    const int64_t N = (int64_t)g->nx * g->ny;
    const int m = g->m;
    const int64_t mm = (int64_t)m * m;
    const int dmin = S.dmin;
    RB_TRY(set_linearise(S, st));
    const double *delta_dir = w.v;  // the update is res[2] * delta_dir
    if (asym) {
        // 3-4. amplitude-normalised backprojection g_A and pair count n_A,
        // one frequency at a time (each with its own 1 / (omega^2 h^2)^2),
        // then v = g_A / n_A on the support
        const int64_t mN = (int64_t)m * N, tot = mN * nf;
        if (o->dtype == RB_F32)
            k_asym_tables<float><<<blocks_for(tot, 256), 256, 0, st>>>(tot, (const float *)w.Gr,
                                                                        (const float *)w.Gi, (float *)w.Hr,
                                                                        (float *)w.Hi, (float *)w.C);
        else
            k_asym_tables<double><<<blocks_for(tot, 256), 256, 0, st>>>(tot, (const double *)w.Gr,
                                                                         (const double *)w.Gi, (double *)w.Hr,
                                                                         (double *)w.Hi, (double *)w.C);
        RB_LAUNCHED();
        if (o->dtype == RB_F32)
            RB_TRY(fill_f32((float *)w.C0, 0.0f, mN, st));
        else
            RB_TRY(fill_f64((double *)w.C0, 0.0, mN, st));
        RB_TRY(fill_f64(w.gA, 0.0, N, st));
        RB_TRY(fill_f64(w.nA, 0.0, N, st));
        const size_t es = dtype_size(o->dtype);
        for (int k = 0; k < nf; ++k) {
            const size_t off = (size_t)k * mN * es;
            RB_TRY(fill_f64(w.gk, 0.0, N, st));
            RB_TRY(fill_f64(w.nk, 0.0, N, st));
            RB_TRY(adjoint_impl(g, (char *)w.Hr + off, (char *)w.Hi + off, nullptr, o->dtype, freqs + k, 1,
                                w.D + (size_t)k * mm * 2, w.W + (size_t)k * mm, w.gk, nullptr, scratch,
                                scratch_bytes, st));
            RB_TRY(hessian_band_impl(g, (char *)w.C + off, w.C0, nullptr, o->dtype, freqs + k, 1, dmin,
                                     reinterpret_cast<int *>(w.zl + (size_t)k * mm), w.nz + k, m * m, w.nk, st));
            const double om = 2.0 * M_PI * freqs[k];
            const double c2 = om * om * g->h * g->h;
            const double sc = 1.0 / (c2 * c2);
            k_asym_accum<<<blocks_for(N, 256), 256, 0, st>>>(N, w.gk, w.nk, sc, sc, w.gA, w.nA);
            RB_LAUNCHED();
        }
        k_asym_direction<<<blocks_for(N, 256), 256, 0, st>>>(N, w.gA, w.nA, w.S, w.v);
        RB_LAUNCHED();
        // 5. exact step length along v
        RB_TRY(forward_impl(g, w.Gr, w.Gi, w.gscale, o->dtype, freqs, nf, w.v, w.Jv, scratch, scratch_bytes,
                            st, dmin));
        k_beta_partial<<<kRB, 256, 0, st>>>(mm * nf, w.W, w.Jv, w.D, w.part);
        RB_LAUNCHED();
        k_beta_final<<<1, 256, 0, st>>>(w.part, kRB, w.res);
        RB_LAUNCHED();
    } else {
        // 3. gradient and Hessian diagonal
        RB_TRY(fill_f64(w.grad, 0.0, N, st));
        RB_TRY(fill_f64(w.hd, 0.0, N, st));
        RB_TRY(adjoint_impl(g, w.Gr, w.Gi, w.gscale, o->dtype, freqs, nf, w.D, w.W, w.grad, nullptr, scratch,
                            scratch_bytes, st));
        RB_TRY(hessian_band_impl(g, w.Gr, w.Gi, w.gscale, o->dtype, freqs, nf, dmin,
                                 reinterpret_cast<int *>(w.zl), w.nz, m * m, w.hd, st));
        RB_TRY(reduce_max_f64(w.hd, w.S, N, w.part, w.hmax, st));
        // 4-5. preconditioned CG from delta = 0
        k_cg_start<<<kRB, 256, 0, st>>>(N, w.grad, w.hd, w.S, w.hmax, o->eps, w.x, w.r, w.z, w.p, w.part);
        RB_LAUNCHED();
        k_cg_rz_final<<<1, 256, 0, st>>>(w.part, kRB, w.cg, 1);
        RB_LAUNCHED();
        for (int it = 0; it < cg_iters; ++it) {
            RB_TRY(forward_impl(g, w.Gr, w.Gi, w.gscale, o->dtype, freqs, nf, w.p, w.Jv, scratch, scratch_bytes,
                                st, dmin));
            // second partial component: <J p, W J p>
            k_beta_partial<<<kRB, 256, 0, st>>>(mm * nf, w.W, w.Jv, w.Jv, w.part);
            RB_LAUNCHED();
            k_cg_alpha<<<1, 256, 0, st>>>(w.part, kRB, w.cg, w.hist, it);
            RB_LAUNCHED();
            if (it + 1 == cg_iters) break;
            RB_TRY(fill_f64(w.q, 0.0, N, st));
            RB_TRY(adjoint_impl(g, w.Gr, w.Gi, w.gscale, o->dtype, freqs, nf, w.Jv, w.W, w.q, nullptr, scratch,
                                scratch_bytes, st));
            k_cg_step<<<kRB, 256, 0, st>>>(N, w.q, w.hd, w.S, w.hmax, o->eps, w.cg, w.x, w.p, w.r, w.z, w.part);
            RB_LAUNCHED();
            k_cg_rz_final<<<1, 256, 0, st>>>(w.part, kRB, w.cg, 0);
            RB_LAUNCHED();
            k_cg_direction<<<blocks_for(N, 256), 256, 0, st>>>(N, w.z, w.cg, w.p);
            RB_LAUNCHED();
        }
        k_cg_last<<<blocks_for(N, 256), 256, 0, st>>>(N, w.cg, w.p, w.x, w.res);
        RB_LAUNCHED();
        delta_dir = w.x;
    }
    RB_TRY(set_update(S, delta_dir, st));
    if (cg_iters > 0 && cg_hist)
        RB_HIP(hipMemcpyAsync(cg_hist, w.hist, sizeof(double) * 2 * cg_iters, hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
    return set_result(S, dc_l2);
}

// Single steps of several problems on one stream, their backprojections'
// contractions in grouped launches.  status[j] receives each problem's
// status; the call returns the first failure.
rb_status invert_grouped(const rb_set_job *jobs, int n, hipStream_t st) {
    std::vector<SetCtx> ctx(n);
    std::vector<AdjTask *> tasks(n);
    for (int j = 0; j < n; ++j) {
        const rb_set_job &J = jobs[j];
        RB_TRY(set_open(ctx[j], J.g, J.t, J.o, J.c_in, J.alpha0, J.freqs_hz, J.nf, J.p_meas, J.c_out, J.ws,
                        J.ws_bytes, false, false));
    }
    for (int j = 0; j < n; ++j) {
        RB_TRY(step_begin(ctx[j], st));
        tasks[j] = &ctx[j].adj;
    }
    RB_TRY(adjoint_run_grouped(tasks.data(), n, st));
    for (int j = 0; j < n; ++j) RB_TRY(step_end(ctx[j], st));
    RB_HIP(hipStreamSynchronize(st));
    rb_status first = RB_OK;
    for (int j = 0; j < n; ++j) {
        const rb_status sj = set_result(ctx[j], jobs[j].dc_l2);
        if (jobs[j].status) *jobs[j].status = sj;
        if (sj != RB_OK && first == RB_OK) first = sj;
    }
    return first;
}

}  // namespace rb

extern "C" {

size_t rb_invert_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int32_t nf, rb_dtype dtype,
                                 int32_t emitter_batch) {
    if (rb::check_trace(g, t) != RB_OK || nf < 1 || nf > RB_MAX_NF) return 0;
    if (dtype < RB_F64 || dtype > RB_F16) return 0;
    return rb::invert_workspace_bytes(g, t, nf, dtype, emitter_batch, false);
}

size_t rb_invert_asymptotic_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int32_t nf,
                                            rb_dtype dtype, int32_t emitter_batch) {
    if (rb::check_trace(g, t) != RB_OK || nf < 1 || nf > RB_MAX_NF) return 0;
    if (dtype != RB_F64 && dtype != RB_F32) return 0;
    return rb::invert_workspace_bytes(g, t, nf, dtype, emitter_batch, false, true);
}

size_t rb_invert_cg_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int32_t nf, rb_dtype dtype,
                                    int32_t emitter_batch) {
    if (rb::check_trace(g, t) != RB_OK || nf < 1 || nf > RB_MAX_NF) return 0;
    if (dtype < RB_F64 || dtype > RB_F16) return 0;
    return rb::invert_workspace_bytes(g, t, nf, dtype, emitter_batch, true);
}

static rb_status check_invert_args(const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o,
                                   const double *c_in, const double *freqs_hz, int32_t nf, const double *p_meas,
                                   double *c_out, void *ws) {
    RB_TRY(rb::check_trace(g, t));
    RB_TRY(rb::check_freqs(freqs_hz, nf));
    RB_CHECK_ARG(o != nullptr, "invert options are NULL");
    RB_CHECK_ARG(o->dtype >= RB_F64 && o->dtype <= RB_F16, "unknown dtype %d", (int)o->dtype);
    RB_CHECK_ARG(o->recv_fraction > 0.0 && o->recv_fraction <= 1.0, "recv_fraction must be in (0, 1]");
    RB_CHECK_ARG(o->outlier_fraction >= 0.0 && o->outlier_fraction < 1.0, "outlier_fraction must be in [0, 1)");
    RB_CHECK_ARG(std::isfinite(o->eps) && o->eps >= 0.0, "eps must be >= 0");
    RB_CHECK_ARG(std::isfinite(o->y_pow), "y_pow must be finite");
    RB_CHECK_ARG(c_in && p_meas && c_out, "c_in/p_meas/c_out are NULL");
    RB_CHECK_ARG(ws != nullptr, "workspace is NULL");
    return RB_OK;
}

rb_status rb_invert_frequency_set(const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o,
                                  const double *c_in, const double *alpha0, const double *freqs_hz, int32_t nf,
                                  const double *p_meas, double *c_out, double *dc_l2, void *ws, size_t ws_bytes,
                                  void *stream) {
    rb::clear_error();
    RB_TRY(check_invert_args(g, t, o, c_in, freqs_hz, nf, p_meas, c_out, ws));
    return rb::invert_impl(g, t, o, c_in, alpha0, freqs_hz, nf, p_meas, 0, c_out, dc_l2, nullptr, ws, ws_bytes,
                           rb::as_stream(stream));
}

rb_status rb_invert_frequency_set_asymptotic(const rb_geometry *g, const rb_trace_opts *t,
                                             const rb_invert_opts *o, const double *c_in, const double *alpha0,
                                             const double *freqs_hz, int32_t nf, const double *p_meas,
                                             double *c_out, double *dc_l2, void *ws, size_t ws_bytes,
                                             void *stream) {
    rb::clear_error();
    RB_TRY(check_invert_args(g, t, o, c_in, freqs_hz, nf, p_meas, c_out, ws));
    if (o->dtype != RB_F64 && o->dtype != RB_F32) {
        rb::set_error("the asymptotic weights need 32- or 64-bit Green's tables (1 / G is unbounded)");
        return RB_EUNSUPPORTED;
    }
    return rb::invert_impl(g, t, o, c_in, alpha0, freqs_hz, nf, p_meas, 0, c_out, dc_l2, nullptr, ws, ws_bytes,
                           rb::as_stream(stream), true);
}

rb_status rb_invert_frequency_set_cg(const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o,
                                     const double *c_in, const double *alpha0, const double *freqs_hz, int32_t nf,
                                     const double *p_meas, int32_t n_iter, double *c_out, double *dc_l2,
                                     double *cg_hist, void *ws, size_t ws_bytes, void *stream) {
    rb::clear_error();
    RB_TRY(check_invert_args(g, t, o, c_in, freqs_hz, nf, p_meas, c_out, ws));
    RB_CHECK_ARG(n_iter >= 1 && n_iter <= RB_MAX_CG_ITERS, "n_iter must be in [1, %d]", RB_MAX_CG_ITERS);
    return rb::invert_impl(g, t, o, c_in, alpha0, freqs_hz, nf, p_meas, n_iter, c_out, dc_l2, cg_hist, ws,
                           ws_bytes, rb::as_stream(stream));
}

rb_status rb_invert_frequency_sets_grouped(const rb_set_job *jobs, int32_t njobs, void *stream) {
    rb::clear_error();
    RB_CHECK_ARG(jobs != nullptr && njobs >= 1 && njobs <= RB_MAX_GROUP, "njobs must be in [1, %d]", RB_MAX_GROUP);
    for (int j = 0; j < njobs; ++j) {
        const rb_set_job &J = jobs[j];
        if (J.status) *J.status = RB_OK;
        const rb_status sj = check_invert_args(J.g, J.t, J.o, J.c_in, J.freqs_hz, J.nf, J.p_meas, J.c_out, J.ws);
        if (sj != RB_OK) {
            if (J.status) *J.status = sj;
            return sj;
        }
    }
    return rb::invert_grouped(jobs, njobs, rb::as_stream(stream));
}

}  // extern "C"
