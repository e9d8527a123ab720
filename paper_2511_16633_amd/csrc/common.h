// Internal helpers shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/rayborn.h"

namespace rb {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
void clear_error();

#define RB_CHECK_ARG(cond, ...)            \
    do {                                   \
        if (!(cond)) {                     \
            ::rb::set_error(__VA_ARGS__);  \
            return RB_EINVAL;              \
        }                                  \
    } while (0)

#define RB_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::rb::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                  \
            return RB_EHIP;                                                       \
        }                                                                         \
    } while (0)

#define RB_LAUNCHED()                                                              \
    do {                                                                           \
        hipError_t e_ = hipGetLastError();                                         \
        if (e_ != hipSuccess) {                                                    \
            ::rb::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                   \
            return RB_EHIP;                                                        \
        }                                                                          \
    } while (0)

#define RB_TRY(expr)                 \
    do {                             \
        rb_status s_ = (expr);       \
        if (s_ != RB_OK) return s_;  \
    } while (0)

// ---------------------------------------------------------------- workspace
// Carves 256-byte aligned sub-buffers out of a caller workspace.  With a
// null base it only measures.
struct Carver {
    char *base;
    size_t cap;
    size_t used = 0;
    Carver(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
    template <typename T>
    T *take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
    bool fits() const { return used <= cap; }
};

inline size_t dtype_size(rb_dtype d) {
    switch (d) {
        case RB_F64: return 8;
        case RB_F32: return 4;
        case RB_BF16: return 2;
        case RB_F16: return 2;
    }
    return 0;
}

rb_status check_geometry(const rb_geometry *g);
rb_status check_trace(const rb_geometry *g, const rb_trace_opts *t);
rb_status check_freqs(const double *f, int32_t nf);
int64_t trace_nmax(const rb_trace_opts *t);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline unsigned blocks_for(int64_t n, int threads) {
    return static_cast<unsigned>((n + threads - 1) / threads);
}

// Workgroups of a launch go to the eight XCDs round-robin by flat id.  This
// bijection on [0, nblk) gives each XCD one contiguous range of logical ids,
// so that workgroups that touch neighbouring data share one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblk) {
    const int64_t q = nblk >> 3, r = nblk & 7, x = b & 7, s = b >> 3;
    return x * q + (x < r ? x : r) + s;
}

// Immediate of s_waitcnt that waits until at most n vector-memory operations
// of the wave are outstanding and leaves the other counters alone (CDNA
// encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).  Direct
// global->LDS loads count here, so this orders them with later LDS reads.
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8); }

// Workgroup barrier that orders LDS accesses only.  Unlike __syncthreads()
// it does not wait for the wave's global loads still in flight (direct
// global->LDS loads filling another buffer are ordered with vmcnt waits).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Fill kernels are used instead of hipMemsetAsync so that a caller may
// capture the library's work into a HIP graph.
rb_status fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st);
rb_status fill_f64(double *p, double v, int64_t n, hipStream_t st);
rb_status fill_f32(float *p, float v, int64_t n, hipStream_t st);

// Deterministic reductions (fixed-order two-level trees).
// out[0] = max over n of in[i] where mask[i] (mask may be null).
rb_status reduce_max_f64(const double *in, const uint8_t *mask, int64_t n, double *partials,
                         double *out, hipStream_t st);
rb_status reduce_max_f32(const float *in, int64_t n, float *partials, float *out,
                         hipStream_t st);
// out[0] = max over n of |in[i]| (0 for an all-zero input).
rb_status reduce_absmax_f64(const double *in, int64_t n, double *partials, double *out, hipStream_t st);

constexpr int kReduceBlocks = 1024;

// Grid/trace parameters passed by value to kernels.
struct GridParams {
    int nx, ny;
    double h, x0, y0;
    double s_bg;
};

// Field value at integer pixel (i, j) with a fixed value outside the grid.
struct SA {
    double s, a;
};

}  // namespace rb
