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
// Every reduction here has a fixed order (per-block trees over a fixed grid,
// then one block), and the outlier selection uses integer keys, so the
// result does not depend on scheduling.
#include <algorithm>
#include <cmath>

#include "born.h"
#include "common.h"
#include "green.h"

namespace rb {

size_t trace_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int batch);
rb_status trace_rays_impl(const rb_geometry *g, const rb_trace_opts *t, const double *slowness,
                          const double *alpha0, const rb_tables *out, void *ws, size_t ws_bytes, hipStream_t st);

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

__device__ __forceinline__ bool selected(int64_t i, int m, int dmin) {
    const int e = (int)(i / m), r = (int)(i - (int64_t)e * m);
    int d = e > r ? e - r : r - e;
    d = d < m - d ? d : m - d;
    return d >= dmin;
}

// Data weights for one frequency per block: receiver selection, then zero the
// kzero selected pairs with the largest |p_meas|^2 (ties to the smaller flat
// index).  The k-th largest key is found by an 8-bit radix select on the
// IEEE bits of |p|^2 (non-negative doubles order like their bit patterns).
constexpr int kWThreads = 1024;
__global__ void __launch_bounds__(kWThreads) k_weights(int m, int dmin, int64_t kzero,
                                                       const double *__restrict__ pmeas,
                                                       double *__restrict__ W) {
    __shared__ unsigned hist[256];
    __shared__ uint64_t s_pref;
    __shared__ int64_t s_rem;
    __shared__ int64_t scan[kWThreads];
    const int k = blockIdx.x, tid = threadIdx.x;
    const int64_t mm = (int64_t)m * m;
    const double *pk = pmeas + 2 * (int64_t)k * mm;
    double *wk = W + (int64_t)k * mm;
    auto key_of = [&](int64_t i) -> uint64_t {
        const double re = pk[2 * i], im = pk[2 * i + 1];
        return (uint64_t)__double_as_longlong(re * re + im * im);
    };
    uint64_t kstar = ~0ull;
    int64_t need = 0;
    if (kzero > 0) {
        if (tid == 0) {
            s_pref = 0;
            s_rem = kzero;
        }
        __syncthreads();
        for (int shift = 56; shift >= 0; shift -= 8) {
            if (tid < 256) hist[tid] = 0;
            __syncthreads();
            const uint64_t pref = s_pref;
            for (int64_t i = tid; i < mm; i += kWThreads) {
                if (!selected(i, m, dmin)) continue;
                const uint64_t key = key_of(i);
                if (shift < 56 && (key >> (shift + 8)) != (pref >> (shift + 8))) continue;
                atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                int64_t rem = s_rem;
                for (int dgt = 255; dgt >= 0; --dgt) {
                    if (rem <= (int64_t)hist[dgt]) {
                        s_pref = pref | ((uint64_t)dgt << shift);
                        break;
                    }
                    rem -= hist[dgt];
                }
                s_rem = rem;
            }
            __syncthreads();
        }
        kstar = s_pref;
        need = s_rem;  // how many keys equal to kstar are zeroed, lowest index first
    }
    // contiguous chunk per thread, so tie ranks follow the flat index
    const int64_t chunk = (mm + kWThreads - 1) / kWThreads;
    const int64_t lo = (int64_t)tid * chunk, hi = std::min<int64_t>(mm, lo + chunk);
    int64_t ties = 0;
    if (kzero > 0)
        for (int64_t i = lo; i < hi; ++i)
            if (selected(i, m, dmin) && key_of(i) == kstar) ++ties;
    scan[tid] = ties;
    __syncthreads();
    if (tid == 0) {
        int64_t acc = 0;
        for (int t = 0; t < kWThreads; ++t) {
            const int64_t v = scan[t];
            scan[t] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int64_t rank = scan[tid];
    for (int64_t i = lo; i < hi; ++i) {
        double w = 0.0;
        if (selected(i, m, dmin)) {
            w = 1.0;
            if (kzero > 0) {
                const uint64_t key = key_of(i);
                if (key > kstar) {
                    w = 0.0;
                } else if (key == kstar) {
                    if (rank < need) w = 0.0;
                    ++rank;
                }
            }
        }
        wk[i] = w;
    }
}

// The zeroed selected pairs of one frequency per block, as (e, r) in flat
// index order (for the banded Hessian diagonal): per-thread counts over
// contiguous chunks, an exclusive scan in thread order, then the writes.
__global__ void __launch_bounds__(kWThreads) k_zero_list(int m, int dmin, const double *__restrict__ W, int zcap,
                                                         int2 *__restrict__ zl, int *__restrict__ nz) {
    __shared__ int64_t scan[kWThreads];
    const int k = blockIdx.x, tid = threadIdx.x;
    const int64_t mm = (int64_t)m * m;
    const double *wk = W + (int64_t)k * mm;
    const int64_t chunk = (mm + kWThreads - 1) / kWThreads;
    const int64_t lo = (int64_t)tid * chunk, hi = std::min<int64_t>(mm, lo + chunk);
    int64_t cnt = 0;
    for (int64_t i = lo; i < hi; ++i)
        if (selected(i, m, dmin) && wk[i] == 0.0) ++cnt;
    scan[tid] = cnt;
    __syncthreads();
    if (tid == 0) {
        int64_t acc = 0;
        for (int t = 0; t < kWThreads; ++t) {
            const int64_t v = scan[t];
            scan[t] = acc;
            acc += v;
        }
        nz[k] = (int)std::min<int64_t>(acc, zcap);
    }
    __syncthreads();
    int64_t pos = scan[tid];
    for (int64_t i = lo; i < hi && pos < zcap; ++i) {
        if (selected(i, m, dmin) && wk[i] == 0.0) {
            const int e = (int)(i / m);
            zl[(int64_t)k * zcap + pos] = make_int2(e, (int)(i - (int64_t)e * m));
            ++pos;
        }
    }
}

// Support: |x| < R - margin and covered by every emitter.
__global__ void k_support(int nx, int ny, double h, double x0, double y0, double rs, int m,
                          const double *__restrict__ T, uint8_t *__restrict__ S) {
    const int64_t N = (int64_t)nx * ny;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t j = p / nx, i = p - j * nx;
    const double px = x0 + (double)i * h, py = y0 + (double)j * h;
    uint8_t ok = (px * px + py * py < rs * rs) ? 1 : 0;
    for (int e = 0; e < m && ok; ++e)
        if (isnan(T[(int64_t)e * N + p])) ok = 0;
    S[p] = ok;
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

struct InvWs {
    double *s, *T, *Trx, *D, *W, *Jv, *grad, *hd, *v, *part, *res, *hmax;
    float *amp, *att, *amp_rx, *att_rx, *gscale;
    void *Gr, *Gi;
    uint8_t *S;
    int2 *zl;   // zeroed pairs [nf][m m]
    int *nz;    // their counts [nf]
    void *scratch;
};

InvWs carve_inv(Carver &c, const rb_geometry *g, int nf, rb_dtype dt) {
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

size_t invert_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int nf, rb_dtype dt, int batch) {
    Carver c(nullptr, 0);
    carve_inv(c, g, nf, dt);
    return c.used + 256 + scratch_need(g, t, nf, dt, batch);
}

rb_status invert_impl(const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o, const double *c_in,
                      const double *alpha0, const double *freqs, int nf, const double *p_meas, double *c_out,
                      double *dc_l2, void *ws, size_t ws_bytes, hipStream_t st) {
    Carver c(ws, ws_bytes);
    InvWs w = carve_inv(c, g, nf, o->dtype);
    if (c.used + 256 + trace_workspace_bytes(g, t, 1) > ws_bytes ||
        c.used + 256 + std::max(adjoint_workspace_bytes(g, nf, o->dtype),
                                forward_workspace_bytes(g, nf, o->dtype)) > ws_bytes) {
        set_error("invert workspace too small (%zu bytes)", ws_bytes);
        return RB_ENOMEM;
    }
    const size_t scratch_bytes = ws_bytes - c.used - 256;
    void *scratch = reinterpret_cast<void *>(((uintptr_t)w.scratch + 255) & ~(uintptr_t)255);
    const int64_t N = (int64_t)g->nx * g->ny;
    const int m = g->m;
    const int64_t mm = (int64_t)m * m;

    // 1. rays, tables and Green's functions in the current model
    k_slowness<<<blocks_for(N, 256), 256, 0, st>>>(c_in, N, w.s);
    RB_LAUNCHED();
    rb_tables tab{w.T, w.amp, w.att, w.Trx, w.amp_rx, w.att_rx};
    RB_TRY(trace_rays_impl(g, t, w.s, alpha0, &tab, scratch, scratch_bytes, st));
    {
        Carver gc(scratch, scratch_bytes);
        float *amax = gc.take<float>(1);
        float *parts = gc.take<float>(kReduceBlocks);
        RB_TRY(build_green_impl(w.T, w.amp, w.att, (int64_t)m * N, freqs, nf, o->y_pow, o->dtype, w.Gr, w.Gi,
                                w.gscale, amax, parts, st));
    }
    // 2. residual and data weights
    GreenParams GP = green_params(freqs, nf, o->y_pow);
    k_residual<<<blocks_for(mm * nf, 256), 256, 0, st>>>(GP, m, w.Trx, w.amp_rx, w.att_rx, p_meas, w.D);
    RB_LAUNCHED();
    const int dmin = (int)std::ceil((1.0 - o->recv_fraction) * 0.5 * m - 1e-9);
    const int64_t n_valid = (int64_t)m * selected_count(m, dmin);
    const int64_t kzero = (int64_t)std::floor(o->outlier_fraction * (double)n_valid);
    k_weights<<<nf, kWThreads, 0, st>>>(m, dmin, kzero, p_meas, w.W);
    RB_LAUNCHED();
    // 3. gradient and Hessian diagonal
    // the Hessian diagonal comes from the band structure of W: the
    // backprojection computes the gradient only
    k_zero_list<<<nf, kWThreads, 0, st>>>(m, dmin, w.W, m * m, w.zl, w.nz);
    RB_LAUNCHED();
    RB_TRY(fill_f64(w.grad, 0.0, N, st));
    RB_TRY(fill_f64(w.hd, 0.0, N, st));
    RB_TRY(adjoint_impl(g, w.Gr, w.Gi, w.gscale, o->dtype, freqs, nf, w.D, w.W, w.grad, nullptr, scratch,
                        scratch_bytes, st));
    RB_TRY(hessian_band_impl(g, w.Gr, w.Gi, w.gscale, o->dtype, freqs, nf, dmin, reinterpret_cast<int *>(w.zl),
                             w.nz, m * m, w.hd, st));
    // 4. diagonally weighted direction on the support
    const double rs = g->ring_radius - g->support_margin;
    k_support<<<blocks_for(N, 256), 256, 0, st>>>(g->nx, g->ny, g->h, g->x0, g->y0, rs, m, w.T, w.S);
    RB_LAUNCHED();
    RB_TRY(reduce_max_f64(w.hd, w.S, N, w.part, w.hmax, st));
    k_direction<<<blocks_for(N, 256), 256, 0, st>>>(N, w.grad, w.hd, w.S, w.hmax, o->eps, w.v);
    RB_LAUNCHED();
    // 5. exact step length along v
    RB_TRY(forward_impl(g, w.Gr, w.Gi, w.gscale, o->dtype, freqs, nf, w.v, w.Jv, scratch, scratch_bytes, st));
    k_beta_partial<<<kRB, 256, 0, st>>>(mm * nf, w.W, w.Jv, w.D, w.part);
    RB_LAUNCHED();
    k_beta_final<<<1, 256, 0, st>>>(w.part, kRB, w.res);
    RB_LAUNCHED();
    // 6. update of 1/c^2 and the update norm
    k_update_partial<<<kRB, 256, 0, st>>>(N, c_in, w.s, w.v, w.res, w.part);
    RB_LAUNCHED();
    k_update_final<<<1, 256, 0, st>>>(w.part, kRB, w.res);
    RB_LAUNCHED();
    k_update_write<<<blocks_for(N, 256), 256, 0, st>>>(N, c_in, w.s, w.v, w.res, c_out);
    RB_LAUNCHED();
    double res[8];
    RB_HIP(hipMemcpyAsync(res, w.res, sizeof(res), hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
    if (res[4] != 0.0) {
        if (dc_l2) *dc_l2 = 0.0;
        set_error("1/c^2 + delta <= 0 at %.0f pixels; model left unchanged", res[4]);
        return RB_ENUMERIC;
    }
    if (dc_l2) *dc_l2 = std::sqrt(res[3]);
    return RB_OK;
}

}  // namespace rb

extern "C" {

size_t rb_invert_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int32_t nf, rb_dtype dtype,
                                 int32_t emitter_batch) {
    if (rb::check_trace(g, t) != RB_OK || nf < 1 || nf > RB_MAX_NF) return 0;
    if (dtype < RB_F64 || dtype > RB_F16) return 0;
    return rb::invert_workspace_bytes(g, t, nf, dtype, emitter_batch);
}

rb_status rb_invert_frequency_set(const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o,
                                  const double *c_in, const double *alpha0, const double *freqs_hz, int32_t nf,
                                  const double *p_meas, double *c_out, double *dc_l2, void *ws, size_t ws_bytes,
                                  void *stream) {
    rb::clear_error();
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
    return rb::invert_impl(g, t, o, c_in, alpha0, freqs_hz, nf, p_meas, c_out, dc_l2, ws, ws_bytes,
                           rb::as_stream(stream));
}

}  // extern "C"
