// Green's-function helpers shared by the build_green and invert sources.
#pragma once
#include "common.h"

namespace rb {

struct GreenParams {
    int nf;
    double f[RB_MAX_NF];
    double rsq[RB_MAX_NF];  // omega^(-1/2)
    double fy[RB_MAX_NF];   // (f / 1 MHz)^y
};

GreenParams green_params(const double *freqs, int nf, double y_pow);

// G at one table entry (T = t, absorption b) and frequency k, with the
// amplitude factor `amag` (a omega^-1/2, or a / max(a) for 16-bit storage):
// the phase is reduced to [0, 1) cycles in FP64 before sincospi.
__device__ __forceinline__ void green_value(const GreenParams &P, int k, double t, double amag, double b,
                                            double &re, double &im) {
    const double cycles = P.f[k] * t + 0.125;
    const double frac = cycles - floor(cycles);
    double sn, cs;
    sincospi(2.0 * frac, &sn, &cs);
    const double mag = amag * exp(-b * P.fy[k]);
    re = mag * cs;
    im = mag * sn;
}

// The same for tables stored in 16 bits (8 or 11 significant bits): the
// phase is reduced to [0, 1) cycles in FP64 as above, then its sine and
// cosine and the magnitude a exp(-b f^y) are taken in FP32 (errors of a few
// 1e-7, far below the 16-bit rounding).
__device__ __forceinline__ void green_value_mag32(const GreenParams &P, int k, double t, float amag, float b,
                                                  double &re, double &im) {
    const double cycles = P.f[k] * t + 0.125;
    const float frac = (float)(cycles - floor(cycles));
    float sn, cs;
    sincospif(2.0f * frac, &sn, &cs);
    const float mag = amag * expf(-b * (float)P.fy[k]);
    re = (double)(mag * cs);
    im = (double)(mag * sn);
}

// Green's tables written by the rasteriser's write pass in place of the
// T/amp/att tables: G [nf][m][N] in FP64, FP32 (scale 1) or BF16 (G /
// omega^-1/2, scale omega^-1/2 per frequency).
struct GreenOut {
    GreenParams P;
    rb_dtype dt;   // RB_F32, RB_F64 or RB_BF16
    void *Gr, *Gi;
};
size_t green_workspace_bytes();
// Tables [n] -> planar G [nf][n] of dtype; scale [nf] (nullable for 32/64-bit).
rb_status build_green_impl(const double *T, const float *amp, const float *att, int64_t n,
                           const double *freqs, int nf, double y_pow, rb_dtype dt, void *G_re, void *G_im,
                           float *scale, float *amp_max_scratch, float *partials, hipStream_t st);

}  // namespace rb
