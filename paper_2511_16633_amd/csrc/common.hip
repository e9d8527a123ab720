// Error reporting, argument checks, fill kernels and deterministic reductions.
#include <cmath>
#include <cstdarg>

#include "common.h"

namespace rb {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

rb_status check_geometry(const rb_geometry *g) {
    RB_CHECK_ARG(g != nullptr, "geometry is NULL");
    RB_CHECK_ARG(g->nx >= 1 && g->ny >= 1, "grid must be at least 1x1 (nx=%d ny=%d)", g->nx, g->ny);
    RB_CHECK_ARG((int64_t)g->nx * g->ny <= (int64_t)1 << 28, "grid too large");
    RB_CHECK_ARG(std::isfinite(g->h) && g->h > 0.0, "h must be positive");
    RB_CHECK_ARG(std::isfinite(g->x0) && std::isfinite(g->y0), "x0/y0 must be finite");
    RB_CHECK_ARG(g->m >= 4 && g->m <= 4096, "m must be in [4, 4096] (m=%d)", g->m);
    RB_CHECK_ARG(std::isfinite(g->ring_radius) && g->ring_radius > 0.0, "ring radius must be positive");
    RB_CHECK_ARG(std::isfinite(g->support_margin), "support margin must be finite");
    RB_CHECK_ARG(std::isfinite(g->c_background) && g->c_background > 0.0, "c_background must be positive");
    return RB_OK;
}

int64_t trace_nmax(const rb_trace_opts *t) { return (int64_t)std::floor(t->tau_max / t->dtau); }

rb_status check_trace(const rb_geometry *g, const rb_trace_opts *t) {
    RB_TRY(check_geometry(g));
    RB_CHECK_ARG(t != nullptr, "trace options are NULL");
    RB_CHECK_ARG(t->n_rays >= 3 && t->n_rays <= 8192, "n_rays must be in [3, 8192]");
    RB_CHECK_ARG(std::isfinite(t->dtau) && t->dtau > 0.0, "dtau must be positive");
    RB_CHECK_ARG(std::isfinite(t->tau_max) && t->tau_max > t->dtau, "tau_max must exceed dtau");
    int64_t nmax = trace_nmax(t);
    // steps are a launch-grid dimension (4 per block, at most 65535 blocks)
    RB_CHECK_ARG(nmax >= 1 && nmax <= 4 * 65535 - 4, "tau_max/dtau gives %lld steps (max 262136)",
                 (long long)nmax);
    RB_CHECK_ARG(std::isfinite(t->j_min), "j_min must be finite");
    return RB_OK;
}

rb_status check_freqs(const double *f, int32_t nf) {
    RB_CHECK_ARG(nf >= 1 && nf <= RB_MAX_NF, "nf must be in [1, %d]", RB_MAX_NF);
    RB_CHECK_ARG(f != nullptr, "freqs_hz is NULL");
    for (int k = 0; k < nf; ++k)
        RB_CHECK_ARG(std::isfinite(f[k]) && f[k] > 0.0, "frequency %d is not positive", k);
    return RB_OK;
}

// ---------------------------------------------------------------- fills
template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

template <typename T>
static rb_status fill(T *p, T v, int64_t n, hipStream_t st) {
    if (n <= 0) return RB_OK;
    unsigned b = blocks_for(n, 256);
    if (b > 8192) b = 8192;
    k_fill<T><<<b, 256, 0, st>>>(p, v, n);
    RB_LAUNCHED();
    return RB_OK;
}

rb_status fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st) { return fill(p, v, n, st); }
rb_status fill_f64(double *p, double v, int64_t n, hipStream_t st) { return fill(p, v, n, st); }
rb_status fill_f32(float *p, float v, int64_t n, hipStream_t st) { return fill(p, v, n, st); }

// ---------------------------------------------------------------- reductions
// max is exact and order-independent, so these are deterministic.
template <typename T, bool ABS = false>
__global__ void k_max_partial(const T *in, const uint8_t *mask, int64_t n, T *partials) {
    __shared__ T sh[256];
    T best = ABS ? (T)0 : -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (!mask || mask[i]) {
            T v = ABS ? fabs(in[i]) : in[i];
            best = v > best ? v : best;
        }
    }
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            T o = sh[threadIdx.x + s];
            if (o > sh[threadIdx.x]) sh[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

// The same for FP32 data read as float4 (16-byte aligned `in`, n4 = n / 4
// vectors), four loads in flight per thread; the n % 4 trailing values are
// taken by block 0.
__global__ void k_max_partial_f32x4(const float4 *__restrict__ in, int64_t n4, const float *__restrict__ tail,
                                    int ntail, float *__restrict__ partials) {
    __shared__ float sh[256];
    float best = -INFINITY;
    auto take = [&](float v) { best = v > best ? v : best; };
    auto take4 = [&](const float4 &v) {
        take(v.x);
        take(v.y);
        take(v.z);
        take(v.w);
    };
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = in[i], b = in[i + stride], c = in[i + 2 * stride], d = in[i + 3 * stride];
        take4(a);
        take4(b);
        take4(c);
        take4(d);
    }
    for (; i < n4; i += stride) take4(in[i]);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) take(tail[threadIdx.x]);
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const float o = sh[threadIdx.x + s];
            if (o > sh[threadIdx.x]) sh[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

template <typename T>
__global__ void k_max_final(const T *partials, int np, T *out) {
    __shared__ T sh[256];
    T best = -INFINITY;
    for (int i = threadIdx.x; i < np; i += 256) best = partials[i] > best ? partials[i] : best;
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s && sh[threadIdx.x + s] > sh[threadIdx.x]) sh[threadIdx.x] = sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

rb_status reduce_max_f64(const double *in, const uint8_t *mask, int64_t n, double *partials,
                         double *out, hipStream_t st) {
    k_max_partial<double><<<kReduceBlocks, 256, 0, st>>>(in, mask, n, partials);
    RB_LAUNCHED();
    k_max_final<double><<<1, 256, 0, st>>>(partials, kReduceBlocks, out);
    RB_LAUNCHED();
    return RB_OK;
}

rb_status reduce_absmax_f64(const double *in, int64_t n, double *partials, double *out, hipStream_t st) {
    k_max_partial<double, true><<<kReduceBlocks, 256, 0, st>>>(in, nullptr, n, partials);
    RB_LAUNCHED();
    k_max_final<double><<<1, 256, 0, st>>>(partials, kReduceBlocks, out);
    RB_LAUNCHED();
    return RB_OK;
}

rb_status reduce_max_f32(const float *in, int64_t n, float *partials, float *out, hipStream_t st) {
    if (((uintptr_t)in & 15) == 0) {
        const int64_t n4 = n / 4;
        k_max_partial_f32x4<<<kReduceBlocks, 256, 0, st>>>(reinterpret_cast<const float4 *>(in), n4, in + 4 * n4,
                                                           (int)(n - 4 * n4), partials);
    } else {
        k_max_partial<float><<<kReduceBlocks, 256, 0, st>>>(in, nullptr, n, partials);
    }
    RB_LAUNCHED();
    k_max_final<float><<<1, 256, 0, st>>>(partials, kReduceBlocks, out);
    RB_LAUNCHED();
    return RB_OK;
}

}  // namespace rb

extern "C" {

const char *rb_status_string(rb_status s) {
    switch (s) {
        case RB_OK: return "ok";
        case RB_EINVAL: return "invalid argument";
        case RB_ENOMEM: return "workspace too small";
        case RB_EHIP: return "HIP runtime error";
        case RB_EUNSUPPORTED: return "unsupported";
        case RB_ENUMERIC: return "non-positive 1/c^2 after update";
    }
    return "unknown status";
}

const char *rb_last_error(void) { return rb::g_err; }

const char *rb_version(void) { return "rayborn 0.1 (gfx950)"; }

}  // extern "C"
