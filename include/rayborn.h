/*
 * rayborn.h - C ABI of the MI355X ray-Born single-step inversion library.
 *
 * The library implements one linearised frequency set of Hessian-free
 * ray-Born inversion for 2-D ring-array sound-speed tomography
 * (arXiv 2511.16633): ray tracing and ray-to-grid tables for the
 * high-frequency Green's functions (Forward Problem section, Eqs. 4-7), the
 * Born forward and weighted adjoint contractions and the diagonally weighted
 * single step (Inverse Problem section, Eqs. 8-10 and the single-step
 * paragraph), the conjugate-gradient solution of the same linear
 * subproblem that the single step replaces, the single step with asymptotic
 * (amplitude-normalised) weights, and the bent-ray time-of-flight
 * inversion that provides the starting model.
 *
 * Conventions shared by every entry point:
 *  - Pointers are DEVICE pointers unless marked [host].  The caller owns and
 *    allocates every buffer; the library allocates no device memory.  Entry
 *    points that need scratch take a caller workspace `ws` of `ws_bytes`
 *    (256-byte aligned) sized by the matching *_workspace_bytes function.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    is asynchronous unless stated; outputs are valid once the stream has
 *    drained.  Entry points hold no global mutable state and may be called
 *    concurrently on different streams with disjoint buffers.
 *  - Grids are [ny][nx] row-major; pixel (i, j) has its centre at
 *    (x0 + i h, y0 + j h); N = nx * ny.  Ring element e (0 <= e < m) sits at
 *    R (cos 2 pi e / m, sin 2 pi e / m).  Outside the grid the medium is
 *    water: slowness 1 / c_background and no absorption.
 *  - Complex data are interleaved (re, im) FP64 pairs; data cubes are
 *    [nf][m (emitter e)][m (receiver r)].
 *  - Green's tables G_re / G_im start on a 16-byte boundary (any hipMalloc
 *    or torch allocation does; an offset view may not): the contractions
 *    read their rows in 16-byte pieces and refuse other pointers with
 *    RB_EINVAL.
 *  - SI units: m, s, Hz, m/s; absorption alpha0 in Np / (m MHz^y).
 *  - Errors: invalid arguments are detected on the host before any work is
 *    enqueued and return RB_EINVAL; a HIP launch/runtime failure returns
 *    RB_EHIP; a workspace too small returns RB_ENOMEM.  rb_last_error()
 *    gives a thread-local message for the last failure.  Nothing aborts.
 */
#ifndef RAYBORN_H
#define RAYBORN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RB_OK = 0,
    RB_EINVAL = -1,       /* invalid argument */
    RB_ENOMEM = -2,       /* workspace too small */
    RB_EHIP = -3,         /* HIP runtime or launch error */
    RB_EUNSUPPORTED = -4, /* valid but unsupported combination */
    RB_ENUMERIC = -5      /* 1/c^2 + delta <= 0 somewhere (update refused) */
} rb_status;

/* Storage type of the Green's tables G and of the contraction operands.
 * RB_F64 accumulates in FP64; the others accumulate in FP32.  RB_BF16 and
 * RB_F16 store G scaled by 1/scale[k] per frequency (see rb_build_green). */
typedef enum { RB_F64 = 0, RB_F32 = 1, RB_BF16 = 2, RB_F16 = 3 } rb_dtype;

typedef struct {
    int32_t nx, ny;        /* grid size, >= 1 each */
    double h, x0, y0;      /* spacing (> 0) and centre of pixel (0, 0) */
    int32_t m;             /* ring elements, 4 <= m <= 4096 */
    double ring_radius;    /* R > 0 */
    double support_margin; /* solution support: |x| < R - margin */
    double c_background;   /* water speed outside the grid, > 0 */
} rb_geometry;

/* Ray fan options.  Travel time tau is the ray parameter; node n of every ray
 * has T = n * dtau exactly.  nmax = floor(tau_max / dtau) steps at most; a
 * ray ends at the first node with |x| > R + 2h.  j_min <= 0 means h / 4. */
typedef struct {
    int32_t n_rays;        /* rays per emitter, 3 <= n_rays <= 8192 */
    double dtau;           /* > 0, s */
    double tau_max;        /* > dtau, s */
    double j_min;          /* floor on the ray-tube width J, m */
} rb_trace_opts;

/* Ray-to-grid tables: travel time T (FP64, NaN where no ray triangle covers
 * the point), amplitude factor a = sqrt(c / (8 pi J)) and absorption
 * integral B (FP32, 0 where uncovered).  Pixel tables are [m][N]
 * (pixel-major per emitter); receiver tables are [m][m] (emitter, element). */
typedef struct {
    double *T;
    float *amp;
    float *att;
    double *T_rx;
    float *amp_rx;
    float *att_rx;
} rb_tables;

typedef struct {
    double recv_fraction;    /* receivers used per emitter, (0, 1]; 0.75 */
    double outlier_fraction; /* largest-|p_meas| fraction zeroed, [0, 1); 0.01 */
    double eps;              /* damping, relative to max Hd on the support; 1e-3 */
    double y_pow;            /* absorption power law exponent y; 1 */
    rb_dtype dtype;          /* storage/contraction type */
} rb_invert_opts;

/* Largest number of frequencies one call accepts. */
#define RB_MAX_NF 16

/*
 * Ray tracing and ray-to-grid tables (Forward Problem: Eqs. 4-7; Discussion:
 * the three stages of tracing the rays, computing their amplitudes and
 * carrying the ray parameters back onto the grid).
 *
 * For every emitter e, a fan of n_rays rays is launched into the inward
 * half-plane (angles theta_e + pi + (j + 1/2 - n_rays/2) pi / n_rays) with
 * |p| = s(x_e) and integrated by classic RK4 in travel time:
 *     dx/dtau = p / s^2,  dp/dtau = grad s / s,  dB/dtau = alpha0 / s,
 * where s and alpha0 are bilinear between pixel centres (water outside).
 * The spreading J = |dx/dpsi| at equal tau is taken from neighbouring rays
 * (central chord / (2 sin dpsi), one-sided chord / (2 sin(dpsi/2)) at the
 * fan edges), giving a = sqrt(c(x) / (8 pi max(J, j_min))).  Each cell of
 * the wavefront mesh is split into two triangles; pixel centres and ring
 * elements inside a triangle (barycentrics >= -1e-12) take the barycentric
 * T, a, B of the first arrival: the candidate with the smallest
 * floor(max(u, 0) 2^F), u = T / dtau the interpolated step index and
 * F = 64 - bits(2 nmax n_rays - 1) - bits(nmax), ties going to the triangle
 * first in (step, ray, triangle) order.
 *
 * slowness: [N] FP64 s = 1/c.  alpha0: [N] FP64 or NULL (no absorption).
 * out: all six table pointers required.  ws: rb_trace_workspace_bytes().
 * The work is split into batches of emitters that fit the workspace.
 */
size_t rb_trace_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t,
                                int32_t emitter_batch);
rb_status rb_trace_rays(const rb_geometry *g, const rb_trace_opts *t,
                        const double *slowness, const double *alpha0,
                        const rb_tables *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Green's tables from ray tables (Eqs. 4-5, high-frequency 2-D Green's
 * function A exp(i[omega T + pi/4]) with A = A_geom A_abs):
 *     G_e(x, f) = a omega^(-1/2) exp(-B (f / 1 MHz)^y) exp(i 2 pi frac(f T + 1/8)),
 * zero where T is NaN.  The phase is reduced in FP64 (cycles, not radians).
 *
 * freqs_hz: [host][nf], 1 <= nf <= RB_MAX_NF, each > 0.
 * G_re, G_im: planar [nf][m][N] of `dtype` (double, float, bf16 or fp16).
 * scale: [nf] FP32 device output (may be NULL for RB_F64 / RB_F32, where it
 * is 1); for RB_BF16 / RB_F16 the stored value is G / scale[k] with
 * scale[k] = max(a) omega_k^(-1/2), so every stored |G| <= 1.
 * ws: rb_green_workspace_bytes() (a few KB, used by the 16-bit types).
 */
size_t rb_green_workspace_bytes(void);
rb_status rb_build_green(const rb_geometry *g, const rb_tables *tab,
                         const double *freqs_hz, int32_t nf, double y_pow, rb_dtype dtype,
                         void *G_re, void *G_im, float *scale, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * Born forward operator (linearised Eq. 1 in q = 1/c^2, s(omega) = 1 in
 * Eq. 2, reciprocity of the Green's function):
 *     d_er(omega) = omega^2 h^2 sum_x G_e(x, omega) G_r(x, omega) delta(x).
 * delta: [N] FP64 perturbation of q.  d_out: [nf][m][m] complex (written,
 * symmetric in e, r).  G as produced by rb_build_green; scale as there
 * (NULL = 1).  ws: rb_forward_workspace_bytes(); with 16-bit tables and
 * m >= 1024 (N a multiple of 8) it includes a copy of G times delta
 * (2 nf m N 16-bit values, rows padded to a multiple of 32 pixels) that
 * the 128 x 128-tile kernel reads.
 */
size_t rb_forward_workspace_bytes(const rb_geometry *g, int32_t nf, rb_dtype dtype);
rb_status rb_born_forward(const rb_geometry *g, const void *G_re, const void *G_im,
                          const float *scale, rb_dtype dtype, const double *freqs_hz,
                          int32_t nf, const double *delta, double *d_out,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * Weighted adjoint (backprojection) and Hessian diagonal (gradient and
 * diagonal of the Gauss-Newton Hessian of Eq. 10 under the data weight W):
 *     grad(x)  += sum_k omega_k^2 h^2 Re sum_{e,r} conj(G_e G_r) W_er d_er,
 *     hdiag(x) += sum_k omega_k^4 h^4 sum_{e,r} W_er |G_e|^2 |G_r|^2.
 * d_res: [nf][m][m] complex; w_data: [nf][m][m] real >= 0.  grad, hdiag:
 * [N] FP64, accumulated into (hdiag may be NULL).  Deterministic: repeated
 * calls give bitwise-identical results.  ws: rb_adjoint_workspace_bytes().
 */
size_t rb_adjoint_workspace_bytes(const rb_geometry *g, int32_t nf, rb_dtype dtype);
rb_status rb_born_adjoint_weighted(const rb_geometry *g, const void *G_re, const void *G_im,
                                   const float *scale, rb_dtype dtype, const double *freqs_hz,
                                   int32_t nf, const double *d_res, const double *w_data,
                                   double *grad, double *hdiag, void *ws, size_t ws_bytes,
                                   void *stream);

/*
 * For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation and arguments as rb_born_adjoint_weighted, with no workspace
 * argument.  Its scratch is one fixed array of RB_NOALLOC_SCRATCH_BYTES per
 * GPU, inside the library, allocated when the library is loaded on that GPU
 * and held until the process ends; the call itself allocates nothing.
 * Problems whose rb_adjoint_workspace_bytes() exceeds that size are refused
 * with RB_ENOMEM before any work is enqueued.  Every call on one GPU shares
 * the array: calls that overlap on one GPU (different streams or threads)
 * race and give undefined results; calls ordered on one stream are safe.
 * Results are bitwise those of rb_born_adjoint_weighted.
 */
#define RB_NOALLOC_SCRATCH_BYTES (64u << 20)
rb_status rb_born_adjoint_weighted_noalloc(const rb_geometry *g, const void *G_re, const void *G_im,
                                           const float *scale, rb_dtype dtype, const double *freqs_hz,
                                           int32_t nf, const double *d_res, const double *w_data,
                                           double *grad, double *hdiag, void *stream);

/*
 * Hessian diagonal of Eq. 10 for the data weights the single step uses
 * (Results: receivers on the opposite part of the ring, the largest values
 * of a frequency set zeroed):
 *     W_er = 1 if d(e, r) >= dmin and (e, r) is not zeroed, else 0,
 *     d(e, r) = min(|e - r|, m - |e - r|),
 *     hdiag(x) += sum_k omega_k^4 h^4 sum_{e,r} W_er |G_e|^2 |G_r|^2,
 * equal to rb_born_adjoint_weighted's hdiag for that W, in O(m) per pixel
 * and frequency (circular band sums) instead of O(m^2).  zeroed: device
 * [nf][zcap] pairs (e, r) of int32, each a selected pair (d(e, r) >= dmin)
 * listed at most once, indices in [0, m) (others are ignored); nzero:
 * device [nf] counts (entries beyond zcap are ignored); zcap = 0 means no
 * zeroed pairs (zeroed and nzero may then be NULL).  hdiag: [N] FP64,
 * accumulated into.  G and scale as for rb_born_adjoint_weighted.
 * Deterministic.  No workspace (m <= 4096 always fits).
 */
rb_status rb_born_hessian_banded(const rb_geometry *g, const void *G_re, const void *G_im,
                                 const float *scale, rb_dtype dtype, const double *freqs_hz,
                                 int32_t nf, int32_t dmin, const int32_t *zeroed,
                                 const int32_t *nzero, int32_t zcap, double *hdiag, void *stream);

/*
 * One linearised frequency set, Hessian-free single step (Inverse Problem
 * section; Results section for the data handling):
 *  1. trace rays in c_in and build the tables and the Green's functions;
 *  2. modelled data p_er = G_e(x_r); residual D = p_meas - p;
 *  3. data weight W = receiver selection (circular index distance
 *     >= ceil((1 - recv_fraction) m / 2)) x outlier zeroing (per frequency,
 *     the floor(outlier_fraction n_valid) selected pairs with the largest
 *     |p_meas|^2, ties to the smaller e*m + r);
 *  4. grad = J^T W D and Hd = diag(J^T W J);
 *  5. v = grad / (Hd + eps max_S Hd) on the support S (|x| < R - margin and
 *     covered by every emitter), 0 elsewhere;
 *  6. beta = Re<J v, W D> / <J v, W J v> (0 if the denominator is 0);
 *  7. c_out = (1/c_in^2 + beta v)^(-1/2) where beta v != 0, c_in elsewhere.
 * c_in, c_out: [N] FP64 (may alias).  alpha0: [N] FP64 or NULL.  p_meas:
 * [nf][m][m] complex.  dc_l2: [host] receives sqrt(sum (c_out - c_in)^2);
 * the call synchronises `stream` to deliver it.  Returns RB_ENUMERIC (and
 * leaves c_out = c_in) if 1/c^2 + delta <= 0 at any updated pixel.
 * ws: rb_invert_workspace_bytes().
 */
size_t rb_invert_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int32_t nf,
                                 rb_dtype dtype, int32_t emitter_batch);
rb_status rb_invert_frequency_set(const rb_geometry *g, const rb_trace_opts *t,
                                  const rb_invert_opts *o, const double *c_in,
                                  const double *alpha0, const double *freqs_hz, int32_t nf,
                                  const double *p_meas, double *c_out, double *dc_l2,
                                  void *ws, size_t ws_bytes, void *stream);

/*
 * The same frequency set with the linearised equation solved by conjugate
 * gradients (Inverse Problem section: the earlier method that solves
 * H delta = -grad F iteratively, about 10-15 iterations per set, each a
 * Hessian action) instead of the single step.  Steps 1-4 and 7 are those of
 * rb_invert_frequency_set; steps 5-6 become n_iter iterations of CG on
 * (J^T W J) delta = J^T W D over the pixels ok = S and Hd + eps max_S Hd > 0
 * (delta = 0 elsewhere), preconditioned by the diagonal Hd + eps max_S Hd,
 * from delta = 0:
 *     r = grad, z = p = r / den;  per iteration i:
 *     alpha_i = r.z / <J p, W J p>;  delta += alpha_i p;
 *     (unless last)  r -= alpha_i J^T W J p;  z = r / den;
 *                    p = z + (r.z)_new / (r.z) p.
 * The first iterate is the single step's beta v.  Once r.z or <J p, W J p>
 * is not positive, every later step is zero.  Cost: n_iter Born forwards
 * and n_iter - 1 weighted adjoints on top of one single step's linearisation.
 * n_iter: 1 <= n_iter <= RB_MAX_CG_ITERS.  cg_hist: [host][2 n_iter] or
 * NULL; receives (alpha_i, (r.z)_i before iteration i) per iteration, both 0
 * after a stop.  ws: rb_invert_cg_workspace_bytes().  Other arguments,
 * outputs and errors as for rb_invert_frequency_set.
 */
#define RB_MAX_CG_ITERS 64
size_t rb_invert_cg_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int32_t nf,
                                    rb_dtype dtype, int32_t emitter_batch);
rb_status rb_invert_frequency_set_cg(const rb_geometry *g, const rb_trace_opts *t,
                                     const rb_invert_opts *o, const double *c_in,
                                     const double *alpha0, const double *freqs_hz, int32_t nf,
                                     const double *p_meas, int32_t n_iter, double *c_out,
                                     double *dc_l2, double *cg_hist, void *ws, size_t ws_bytes,
                                     void *stream);

/*
 * One frequency set of several independent problems (jobs of different ring
 * sizes, grids and contraction types), batched: every job's single step as
 * rb_invert_frequency_set computes it, all on one stream, with the
 * backprojection contractions of the jobs grouped into shared launches - a
 * flat grid of (job, frequency, pixel tile) work items, one launch per
 * contraction type for up to 8 jobs - so that small problems fill the GPU
 * together (the serving loop's batched form of the Inverse Problem
 * section's single step).  Each job's result is bitwise the one
 * rb_invert_frequency_set gives it alone: its work items compute exactly
 * what the single-job launch computes, and every reduction keeps its order.
 * Each rb_set_job holds that call's arguments (ws: the job's own workspace
 * of rb_invert_workspace_bytes; jobs may not share workspaces or outputs);
 * status [host], if not NULL, receives the job's own status (RB_ENUMERIC
 * leaves that job's c_out = c_in).  The call synchronises the stream and
 * returns the first failure, RB_OK if none.  1 <= njobs <= RB_MAX_GROUP.
 */
#define RB_MAX_GROUP 256
typedef struct {
    const rb_geometry *g;
    const rb_trace_opts *t;
    const rb_invert_opts *o;
    const double *c_in;
    const double *alpha0;
    const double *freqs_hz;   /* [host][nf] */
    int32_t nf;
    const double *p_meas;
    double *c_out;
    double *dc_l2;            /* [host] out */
    rb_status *status;        /* [host] out, or NULL */
    void *ws;
    size_t ws_bytes;
} rb_set_job;
rb_status rb_invert_frequency_sets_grouped(const rb_set_job *jobs, int32_t njobs, void *stream);

/*
 * The frequency set with asymptotic (amplitude-normalised) weights in place
 * of the Hessian-diagonal weight (single-step paragraph: weights that
 * diagonalise the Hessian, here in their ray-Born asymptotic form; the
 * cited reference's exact weights are not in the paper).  Steps 1-3 and 6-7
 * are those of rb_invert_frequency_set; the direction is the W-weighted mean
 * of the per-pair single-pixel estimates D_er / (omega^2 h^2 G_e(x) G_r(x)):
 *     g_A(x) = sum_k Re sum_{e,r} W_er D_er / (omega_k^2 h^2 G_e(x) G_r(x)),
 *     n_A(x) = sum_k sum_{e,r} W_er [G_e(x) != 0] [G_r(x) != 0],
 *     v(x)   = g_A(x) / n_A(x) on the support S where n_A > 0, 0 elsewhere,
 * then beta = Re<J v, W D> / <J v, W J v> and the update as there.  For
 * Born data of a single pixel's perturbation, v at that pixel is the
 * perturbation itself.  Costs one backprojection and one banded pair count
 * per frequency on the tables H = G / |G|^2 and [G != 0].  dtype must be
 * RB_F64 or RB_F32 (RB_EUNSUPPORTED otherwise: 1 / G is unbounded).
 * ws: rb_invert_asymptotic_workspace_bytes().  Other arguments, outputs and
 * errors as for rb_invert_frequency_set.
 */
size_t rb_invert_asymptotic_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t,
                                            int32_t nf, rb_dtype dtype, int32_t emitter_batch);
rb_status rb_invert_frequency_set_asymptotic(const rb_geometry *g, const rb_trace_opts *t,
                                             const rb_invert_opts *o, const double *c_in,
                                             const double *alpha0, const double *freqs_hz,
                                             int32_t nf, const double *p_meas, double *c_out,
                                             double *dc_l2, void *ws, size_t ws_bytes, void *stream);

/*
 * Starting model by bent-ray time-of-flight (ToF) inversion (Results
 * section: the ray-Born sweep starts from a low-resolution image from three
 * iterations of a ToF-based method that fits measured ToFs with ToFs
 * modelled along rays; Discussion: ray linking).  Per iteration:
 *  1. trace rays in c (s = 1/c, no absorption); the modelled ToF T_er is the
 *     first-arrival time at element r (the T_rx table of rb_trace_rays);
 *  2. linking path of (e, r): the first-arrival triangle at r, of cell
 *     (n, j), gives the step index u and the weight w of ray j + 1
 *     (triangle (P[n][j], P[n][j+1], P[n+1][j+1]): w = lb + lc; triangle
 *     (P[n][j], P[n+1][j+1], P[n+1][j]): w = lb); the path is ray j with
 *     weight 1 - w plus ray j + 1 with weight w, each from the emitter to
 *     parameter u (nodes 0 .. floor(u), then the point at frac(u) along
 *     the next segment);
 *  3. used pairs: circular index distance >= ceil((1 - recv_fraction) m / 2),
 *     T_meas finite and r covered; residual dT = T_meas - T on them;
 *  4. Fermat linearisation dT = L ds: L[er][p] = sum over the path's points
 *     of (path weight) x (half the two adjacent segment lengths) x (bilinear
 *     weight of pixel centre p at the point);
 *  5. g = L^T dT, ray density C = L^T 1; on S (|x| < R - margin and C > 0)
 *     v = g / (C + eps max_S C), 0 elsewhere;
 *  6. beta = <L v, dT> / <L v, L v> (0 if the denominator is 0);
 *     s += beta v, c = 1/s where beta v != 0.
 * o: recv_fraction and eps are used (the other fields are ignored).
 * c_in, c_out: [N] FP64 m/s (may alias).  T_meas: [m][m] FP64 seconds,
 * NaN where no ToF was measured.  n_iter: 1 .. 64.  hist: [host][2 n_iter]
 * or NULL; receives (rms dT over the used pairs before the update, beta)
 * per iteration.  The call synchronises `stream` once per iteration.
 * Every emitter's fan stays resident: ws: rb_tof_workspace_bytes() (about
 * the trace workspace of one batch of all m emitters).  The back-projection
 * sums in 64-bit fixed point (integer atomics, exact and order-independent;
 * contributions rounded to 2^-60 of a bound on a pixel's total), so
 * repeated calls give bitwise-identical results.  Returns RB_ENUMERIC,
 * leaving c_out unwritten, if an update would make s <= 0 somewhere.
 */
size_t rb_tof_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t);
rb_status rb_tof_invert(const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o,
                        const double *c_in, const double *T_meas, int32_t n_iter, double *c_out,
                        double *hist, void *ws, size_t ws_bytes, void *stream);

/* Static description of a status code. */
const char *rb_status_string(rb_status s);
/* Thread-local detail of the last failure on this thread ("" if none). */
const char *rb_last_error(void);
/* Library version string. */
const char *rb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RAYBORN_H */
