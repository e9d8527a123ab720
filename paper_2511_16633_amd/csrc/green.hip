// Green's tables from the ray tables (paper Eqs. 4-5).
//
//   G_e(x, f) = a omega^(-1/2) exp(-B (f / 1 MHz)^y) exp(i 2 pi frac(f T + 1/8))
//
// An HBM-streaming elementwise kernel: each lane reads one (T, a, B) table
// entry (16 bytes) once and writes the nf frequencies of the set, so the
// tables are read once per frequency set rather than once per frequency.
// The phase is reduced to [0, 1) cycles in FP64 before sincospi, and every
// value is computed in FP64 and rounded once to the storage type, except
// that 16-bit tables take the magnitude a exp(-B f^y) in FP32.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "green.h"

namespace rb {
namespace {

template <typename S>
__device__ __forceinline__ S store_cast(double v);
template <>
__device__ __forceinline__ double store_cast<double>(double v) { return v; }
template <>
__device__ __forceinline__ float store_cast<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ __hip_bfloat16 store_cast<__hip_bfloat16>(double v) {
    return __float2bfloat16((float)v);
}
template <>
__device__ __forceinline__ __half store_cast<__half>(double v) { return __float2half((float)v); }

template <typename S, bool SCALED>
__global__ void __launch_bounds__(256) k_green(GreenParams P, const double *__restrict__ T,
                                               const float *__restrict__ amp, const float *__restrict__ att,
                                               int64_t n, const float *__restrict__ amp_max,
                                               S *__restrict__ Gr, S *__restrict__ Gi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = T[i];
    const bool cov = !isnan(t);
    const double a = (double)amp[i], b = (double)att[i];
    const double inv_amax = SCALED ? 1.0 / (double)amp_max[0] : 1.0;
    for (int k = 0; k < P.nf; ++k) {
        double re = 0.0, im = 0.0;
        // 16-bit storage holds G / (max(a) omega^-1/2): |stored| <= 1.  The
        // phase is reduced in FP64; its sine, cosine and the magnitude are
        // taken in FP32 (the table they are rounded to keeps 8 or 11 bits).
        if (cov) {
            if (SCALED)
                green_value_mag32(P, k, t, (float)(a * inv_amax), (float)b, re, im);
            else
                green_value(P, k, t, a * P.rsq[k], b, re, im);
        }
        Gr[(int64_t)k * n + i] = store_cast<S>(re);
        Gi[(int64_t)k * n + i] = store_cast<S>(im);
    }
}

__global__ void k_scales(GreenParams P, const float *__restrict__ amp_max, float *__restrict__ scale,
                         int scaled) {
    const int k = threadIdx.x;
    if (k < P.nf) scale[k] = scaled ? (float)((double)amp_max[0] * P.rsq[k]) : 1.0f;
}

}  // namespace

GreenParams green_params(const double *freqs, int nf, double y_pow) {
    GreenParams P;
    P.nf = nf;
    for (int k = 0; k < nf; ++k) {
        P.f[k] = freqs[k];
        P.rsq[k] = std::pow(2.0 * M_PI * freqs[k], -0.5);
        P.fy[k] = std::pow(freqs[k] * 1e-6, y_pow);
    }
    return P;
}

size_t green_workspace_bytes() { return 256 * 2 + 4 * (kReduceBlocks + 1) + 256; }

rb_status build_green_impl(const double *T, const float *amp, const float *att, int64_t n,
                           const double *freqs, int nf, double y_pow, rb_dtype dt, void *G_re, void *G_im,
                           float *scale, float *amp_max_scratch, float *partials, hipStream_t st) {
    GreenParams P = green_params(freqs, nf, y_pow);
    const bool scaled = (dt == RB_BF16 || dt == RB_F16);
    if (scaled) {
        RB_TRY(reduce_max_f32(amp, n, partials, amp_max_scratch, st));
    }
    const unsigned nb = blocks_for(n, 256);
    switch (dt) {
        case RB_F64:
            k_green<double, false><<<nb, 256, 0, st>>>(P, T, amp, att, n, nullptr, (double *)G_re,
                                                       (double *)G_im);
            break;
        case RB_F32:
            k_green<float, false><<<nb, 256, 0, st>>>(P, T, amp, att, n, nullptr, (float *)G_re,
                                                      (float *)G_im);
            break;
        case RB_BF16:
            k_green<__hip_bfloat16, true><<<nb, 256, 0, st>>>(P, T, amp, att, n, amp_max_scratch,
                                                              (__hip_bfloat16 *)G_re, (__hip_bfloat16 *)G_im);
            break;
        case RB_F16:
            k_green<__half, true><<<nb, 256, 0, st>>>(P, T, amp, att, n, amp_max_scratch, (__half *)G_re,
                                                      (__half *)G_im);
            break;
    }
    RB_LAUNCHED();
    if (scale) {
        k_scales<<<1, 32, 0, st>>>(P, amp_max_scratch, scale, scaled ? 1 : 0);
        RB_LAUNCHED();
    }
    return RB_OK;
}

}  // namespace rb

extern "C" size_t rb_green_workspace_bytes(void) { return rb::green_workspace_bytes(); }

extern "C" rb_status rb_build_green(const rb_geometry *g, const rb_tables *tab, const double *freqs_hz,
                                    int32_t nf, double y_pow, rb_dtype dtype, void *G_re, void *G_im,
                                    float *scale, void *ws, size_t ws_bytes, void *stream) {
    rb::clear_error();
    RB_TRY(rb::check_geometry(g));
    RB_TRY(rb::check_freqs(freqs_hz, nf));
    RB_CHECK_ARG(tab && tab->T && tab->amp && tab->att, "tables are NULL");
    RB_CHECK_ARG(G_re && G_im, "G_re/G_im are NULL");
    RB_CHECK_ARG(dtype >= RB_F64 && dtype <= RB_F16, "unknown dtype %d", (int)dtype);
    RB_CHECK_ARG(std::isfinite(y_pow), "y_pow must be finite");
    const bool scaled = (dtype == RB_BF16 || dtype == RB_F16);
    RB_CHECK_ARG(!scaled || scale != nullptr, "scale is required for 16-bit storage");
    RB_CHECK_ARG(!scaled || ws != nullptr, "workspace is required for 16-bit storage");
    float *amax = nullptr, *partials = nullptr;
    if (scaled) {
        if (ws_bytes < rb::green_workspace_bytes()) {
            rb::set_error("green workspace too small: need %zu bytes", rb::green_workspace_bytes());
            return RB_ENOMEM;
        }
        rb::Carver c(ws, ws_bytes);
        amax = c.take<float>(1);
        partials = c.take<float>(rb::kReduceBlocks);
    }
    const int64_t n = (int64_t)g->m * g->nx * g->ny;
    return rb::build_green_impl(tab->T, tab->amp, tab->att, n, freqs_hz, nf, y_pow, dtype, G_re, G_im,
                                scale, amax, partials, rb::as_stream(stream));
}
