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
size_t green_workspace_bytes();
// Tables [n] -> planar G [nf][n] of dtype; scale [nf] (nullable for 32/64-bit).
rb_status build_green_impl(const double *T, const float *amp, const float *att, int64_t n,
                           const double *freqs, int nf, double y_pow, rb_dtype dt, void *G_re, void *G_im,
                           float *scale, float *amp_max_scratch, float *partials, hipStream_t st);

}  // namespace rb
