// Born contraction kernels (adjoint.hip, forward.hip, hessian.hip): parameters and host
// entry points shared with the inversion driver.
#pragma once
#include "common.h"

namespace rb {

struct AdjParams {
    int m, mp, nb, nf;
    int64_t N;
    double cg[RB_MAX_NF];  // omega^2 h^2
    double ch[RB_MAX_NF];  // omega^4 h^4
};

// One problem's backprojection as the contraction kernel sees it, for
// launches that group several problems: its parameters, its tables and
// prepared operands, its per-frequency partial sums, its pixel tiles per
// frequency, its first flat workgroup in the launch and how many workgroups
// split the emitter passes of one pixel tile.
struct AdjItem {
    AdjParams P;
    const void *Gr, *Gi, *Ar, *Ai, *Wt;
    const uint8_t *flags;
    const float *gscale, *ascale;
    double *pg, *ph;
    int ntiles, begin;
    int npg;   // emitter-pass groups per pixel tile, each a workgroup of its own (partials [nf][npg][N])
};
constexpr int kAdjGroupMax = 8;   // problems per grouped launch (kernel-argument size)
struct AdjGroup {
    int n;
    AdjItem item[kAdjGroupMax];
};

// A prepared backprojection (operands and block flags written on the
// stream), ready for its contraction kernel alone or grouped with others.
struct AdjTask {
    AdjItem item;
    rb_dtype dt;
    double *grad, *hdiag;
};

struct FwdParams {
    int m, mp, nf, ntl, ntri, nsplit;
    int dmin;              // >= 32: diagonal 32 x 32 blocks need not be computed
    int64_t N, kchunk;
    double cg[RB_MAX_NF];  // omega^2 h^2
};

size_t adjoint_workspace_bytes(const rb_geometry *g, int nf, rb_dtype dt);
size_t forward_workspace_bytes(const rb_geometry *g, int nf, rb_dtype dt);

// grad/hdiag += (see rb_born_adjoint_weighted); gscale may be null for 32/64-bit.
rb_status adjoint_impl(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                       rb_dtype dt, const double *freqs, int nf, const double *d_res, const double *w_data,
                       double *grad, double *hdiag, void *ws, size_t ws_bytes, hipStream_t st);
// The same as adjoint_impl in two parts: the operand preparation, then the
// contraction and the frequency sum.  adjoint_run_grouped runs the second
// part of several prepared problems, with one contraction launch per
// contraction type (up to kAdjGroupMax problems each); every problem's result
// is bitwise that of adjoint_impl.  The f64 type is prepared and run alone.
rb_status adjoint_prepare(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                          rb_dtype dt, const double *freqs, int nf, const double *d_res, const double *w_data,
                          double *grad, double *hdiag, void *ws, size_t ws_bytes, hipStream_t st, AdjTask *task);
rb_status adjoint_run(const AdjTask &task, hipStream_t st);
rb_status adjoint_run_grouped(AdjTask *const *tasks, int n, hipStream_t st);
// d_out = J delta, [nf][m][m] complex.  With dmin >= 32 (a caller that
// weights every pair of circular index distance below dmin by zero) the
// 32/16-bit kernels may return 0 for the pairs of a diagonal 32 x 32 block,
// all of which lie below that distance.
rb_status forward_impl(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                       rb_dtype dt, const double *freqs, int nf, const double *delta, double *d_out, void *ws,
                       size_t ws_bytes, hipStream_t st, int dmin = 0);

// hdiag += Hessian diagonal for band-selection weights with zeroed pairs
// (see rb_born_hessian_banded); zeroed: [nf][zcap] (e, r), nzero: [nf].
rb_status hessian_band_impl(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                            rb_dtype dt, const double *freqs, int nf, int dmin, const int *zeroed,
                            const int *nzero, int zcap, double *hdiag, hipStream_t st);

// Argument checks shared by the contraction entry points.
rb_status check_contraction(const rb_geometry *g, const void *G_re, const void *G_im, const float *scale,
                            rb_dtype dt, const double *freqs, int32_t nf);

}  // namespace rb
