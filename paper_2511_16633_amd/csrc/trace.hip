// Ray tracing and ray-to-grid tables.
//
// Model (paper, Forward Problem section): the travel time T solves the
// Eikonal equation (Eq. 6), integrated along rays with T itself as the ray
// parameter; the amplitude follows from the Transport equation (Eq. 7) via
// the ray-tube width J from neighbouring rays; absorption accumulates along
// each ray (Eq. 5).  The tables are formed on the wavefront mesh
// (Discussion: "back-propagation of ray parameters") by first-arrival
// barycentric interpolation.
//
// GPU design:
//  * one lane per ray, classic RK4 in FP64; the slowness and absorption maps
//    are packed into one 16-byte (s, alpha0) record per pixel so a bilinear
//    corner is one load, served from L2/MALL (a 480x480 map is 3.7 MB);
//  * wavefront nodes are stored [emitter][step][ray] so the lanes of a wave
//    write consecutive addresses at every step;
//  * first arrival without floating-point atomics: pass 1 takes an integer
//    atomicMin on an order-preserving 64-bit image of T, pass 2 an atomicMin
//    on the (step, ray, triangle) index among the triangles that attain it,
//    pass 3 recomputes the winner's barycentrics per point.  The result is
//    independent of scheduling.
#include <cmath>

#include "common.h"

namespace rb {
namespace {

struct TP {
    int nx, ny;
    double h, x0, y0;
    int m;
    double R, s_bg;
    int nr;            // rays per emitter
    double dtau;
    int nmax;
    double rdie2;      // (R + 2h)^2
    double j_min;
    double bary_tol;
    double two_sin_full, two_sin_half;
    int e0, ne;        // emitter batch
};

__device__ __forceinline__ double2 corner(const double2 *__restrict__ sa, const TP &P, long i, long j) {
    if (i < 0 || j < 0 || i >= P.nx || j >= P.ny) return make_double2(P.s_bg, 0.0);
    return sa[(size_t)j * (size_t)P.nx + (size_t)i];
}

// Bilinear slowness s with its exact patch gradient, and bilinear alpha0.
__device__ __forceinline__ void field(const double2 *__restrict__ sa, const TP &P, double x, double y,
                                      double &s, double &gx, double &gy, double &a) {
    double u = (x - P.x0) / P.h;
    double v = (y - P.y0) / P.h;
    double fi = floor(u), fj = floor(v);
    if (!(fi >= -1.0 && fi <= (double)P.nx && fj >= -1.0 && fj <= (double)P.ny)) {
        s = P.s_bg; gx = 0.0; gy = 0.0; a = 0.0;
        return;
    }
    long i = (long)fi, j = (long)fj;
    double fu = u - fi, fv = v - fj;
    double2 c00 = corner(sa, P, i, j), c10 = corner(sa, P, i + 1, j);
    double2 c01 = corner(sa, P, i, j + 1), c11 = corner(sa, P, i + 1, j + 1);
    double dx0 = c10.x - c00.x, dx1 = c11.x - c01.x;
    double s0 = c00.x + fu * dx0;
    double s1 = c01.x + fu * dx1;
    s = s0 + fv * (s1 - s0);
    gx = (dx0 + fv * (dx1 - dx0)) / P.h;
    gy = (s1 - s0) / P.h;
    double a0 = c00.y + fu * (c10.y - c00.y);
    double a1 = c01.y + fu * (c11.y - c01.y);
    a = a0 + fv * (a1 - a0);
}

__device__ __forceinline__ void rhs(const double2 *__restrict__ sa, const TP &P, const double st[5],
                                    double d[5]) {
    double s, gx, gy, a;
    field(sa, P, st[0], st[1], s, gx, gy, a);
    double s2 = s * s;
    d[0] = st[2] / s2;
    d[1] = st[3] / s2;
    d[2] = gx / s;
    d[3] = gy / s;
    d[4] = a / s;
}

__global__ void k_pack(const double *__restrict__ s, const double *__restrict__ alpha, int64_t n,
                       double2 *__restrict__ sa) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) sa[i] = make_double2(s[i], alpha ? alpha[i] : 0.0);
}

// One lane per ray: RK4 in travel time, nodes stored [eb][n][j].
__global__ void __launch_bounds__(128) k_trace(TP P, const double2 *__restrict__ sa, double *__restrict__ X,
                                               double *__restrict__ Y, double *__restrict__ Bn,
                                               int *__restrict__ L) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int eb = blockIdx.y;
    if (j >= P.nr || eb >= P.ne) return;
    const int e = P.e0 + eb;
    const double theta = 2.0 * M_PI * (double)e / (double)P.m;
    const double xe = P.R * cos(theta), ye = P.R * sin(theta);
    const double dpsi = M_PI / (double)P.nr;
    double se, gx, gy, av;
    field(sa, P, xe, ye, se, gx, gy, av);
    const double psi = theta + M_PI + ((double)j + 0.5 - 0.5 * (double)P.nr) * dpsi;
    double st[5] = {xe, ye, se * cos(psi), se * sin(psi), 0.0};
    const size_t base = (size_t)eb * (size_t)(P.nmax + 1) * P.nr + j;
    X[base] = st[0];
    Y[base] = st[1];
    Bn[base] = 0.0;
    const double dt = P.dtau, hdt = 0.5 * dt, sixth = dt / 6.0;
    int last = P.nmax;
    for (int n = 0; n < P.nmax; ++n) {
        double k1[5], k2[5], k3[5], k4[5], t[5];
        rhs(sa, P, st, k1);
#pragma unroll
        for (int q = 0; q < 5; ++q) t[q] = st[q] + hdt * k1[q];
        rhs(sa, P, t, k2);
#pragma unroll
        for (int q = 0; q < 5; ++q) t[q] = st[q] + hdt * k2[q];
        rhs(sa, P, t, k3);
#pragma unroll
        for (int q = 0; q < 5; ++q) t[q] = st[q] + dt * k3[q];
        rhs(sa, P, t, k4);
#pragma unroll
        for (int q = 0; q < 5; ++q) st[q] = st[q] + sixth * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
        size_t k = base + (size_t)(n + 1) * P.nr;
        X[k] = st[0];
        Y[k] = st[1];
        Bn[k] = st[4];
        if (st[0] * st[0] + st[1] * st[1] > P.rdie2) {
            last = n + 1;
            break;
        }
    }
    L[(size_t)eb * P.nr + j] = last;
}

// Ray-tube width from neighbouring rays at equal travel time, and the
// amplitude factor a = sqrt(c / (8 pi max(J, j_min))).
__global__ void k_spread(TP P, const double2 *__restrict__ sa, const double *__restrict__ X,
                         const double *__restrict__ Y, const int *__restrict__ L,
                         double *__restrict__ AMP) {
    const int64_t per = (int64_t)(P.nmax + 1) * P.nr;
    const int64_t tot = per * P.ne;
    const double eight_pi = 8.0 * M_PI;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int eb = (int)(idx / per);
        const int64_t rem = idx - (int64_t)eb * per;
        const int n = (int)(rem / P.nr);
        const int j = (int)(rem - (int64_t)n * P.nr);
        const int *Le = L + (size_t)eb * P.nr;
        if (n > Le[j]) continue;
        const size_t k = (size_t)idx;
        const bool lo = (j > 0 && n <= Le[j - 1]);
        const bool hi = (j + 1 < P.nr && n <= Le[j + 1]);
        double Jv = 0.0, dx, dy;
        if (lo && hi) {
            dx = X[k + 1] - X[k - 1];
            dy = Y[k + 1] - Y[k - 1];
            Jv = sqrt(dx * dx + dy * dy) / P.two_sin_full;
        } else if (hi) {
            dx = X[k + 1] - X[k];
            dy = Y[k + 1] - Y[k];
            Jv = sqrt(dx * dx + dy * dy) / P.two_sin_half;
        } else if (lo) {
            dx = X[k] - X[k - 1];
            dy = Y[k] - Y[k - 1];
            Jv = sqrt(dx * dx + dy * dy) / P.two_sin_half;
        }
        if (Jv < P.j_min) Jv = P.j_min;
        double s, gx, gy, av;
        field(sa, P, X[k], Y[k], s, gx, gy, av);
        AMP[k] = sqrt((1.0 / s) / (eight_pi * Jv));
    }
}

// Order-preserving image of a double in uint64 (after turning -0 into +0).
__device__ __forceinline__ uint64_t order_key(double t) {
    t = t + 0.0;
    uint64_t b = (uint64_t)__double_as_longlong(t);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

struct Tri {
    double ax, ay, e1x, e1y, e2x, e2y, det;
    double xmin, xmax, ymin, ymax;
};

__device__ __forceinline__ bool make_tri(double ax, double ay, double bx, double by, double cx, double cy,
                                         Tri &t) {
    t.ax = ax; t.ay = ay;
    t.e1x = bx - ax; t.e1y = by - ay;
    t.e2x = cx - ax; t.e2y = cy - ay;
    t.det = t.e1x * t.e2y - t.e1y * t.e2x;
    if (t.det == 0.0) return false;
    t.xmin = fmin(ax, fmin(bx, cx)); t.xmax = fmax(ax, fmax(bx, cx));
    t.ymin = fmin(ay, fmin(by, cy)); t.ymax = fmax(ay, fmax(by, cy));
    return true;
}

// barycentric test at (qx, qy); returns false when outside
__device__ __forceinline__ bool bary(const Tri &t, double px, double py, double tol, double &la, double &lb,
                                     double &lc) {
    double qx = px - t.ax, qy = py - t.ay;
    lb = (qx * t.e2y - qy * t.e2x) / t.det;
    lc = (t.e1x * qy - t.e1y * qx) / t.det;
    la = (1.0 - lb) - lc;
    return !(la < tol || lb < tol || lc < tol);
}

// Vertices of triangle `tri` of cell (n, j) in node indices.
__device__ __forceinline__ void tri_nodes(int64_t base, int n, int j, int nr, int tri, int64_t &ka,
                                          int64_t &kb, int64_t &kc, int &na, int &nb, int &nc) {
    const int64_t k00 = base + (int64_t)n * nr + j, k10 = k00 + 1;
    const int64_t k01 = k00 + nr, k11 = k01 + 1;
    if (tri == 0) {
        ka = k00; kb = k10; kc = k11; na = n; nb = n; nc = n + 1;
    } else {
        ka = k00; kb = k11; kc = k01; na = n; nb = n + 1; nc = n + 1;
    }
}

// Receivers that may lie in a triangle's bounding box: a conservative index
// range around the ring, or the whole ring when the box contains the centre.
__device__ __forceinline__ bool rx_range(const TP &P, const Tri &t, int &rlo, int &rhi) {
    double dxm = t.xmin > 0.0 ? t.xmin : (t.xmax < 0.0 ? -t.xmax : 0.0);
    double dym = t.ymin > 0.0 ? t.ymin : (t.ymax < 0.0 ? -t.ymax : 0.0);
    double dmin = sqrt(dxm * dxm + dym * dym);
    double dmax = sqrt(fmax(t.xmin * t.xmin, t.xmax * t.xmax) + fmax(t.ymin * t.ymin, t.ymax * t.ymax));
    if (!(dmin >= 0.0) || !(dmax >= 0.0)) return false;  // NaN nodes: nothing to test
    if (dmin > P.R * (1.0 + 1e-9) || dmax < P.R * (1.0 - 1e-9)) return false;
    if (dmin <= 0.0) {
        rlo = 0; rhi = P.m - 1;
        return true;
    }
    double cx = 0.5 * (t.xmin + t.xmax), cy = 0.5 * (t.ymin + t.ymax);
    double th = atan2(cy, cx);
    double lo = 0.0, hi = 0.0;
    double xs[2] = {t.xmin, t.xmax}, ys[2] = {t.ymin, t.ymax};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            double rel = atan2(cx * ys[b] - cy * xs[a], cx * xs[a] + cy * ys[b]);
            lo = fmin(lo, rel);
            hi = fmax(hi, rel);
        }
    double w = 2.0 * M_PI / (double)P.m;
    const double flo = floor((th + lo) / w) - 1.0, fhi = ceil((th + hi) / w) + 1.0;
    if (!(fhi - flo + 1.0 < (double)P.m) || !(flo >= -2.0 * P.m) || !(fhi <= 2.0 * P.m)) {
        rlo = 0; rhi = P.m - 1;   // whole ring (also catches non-finite angles)
        return true;
    }
    rlo = (int)flo;
    rhi = (int)fhi;
    return true;
}

__device__ __forceinline__ void rx_pos(const TP &P, int r, double &x, double &y) {
    double th = 2.0 * M_PI * (double)r / (double)P.m;
    x = P.R * cos(th);
    y = P.R * sin(th);
}

// Pass 1 (mode 0): atomicMin of the T key.  Pass 2 (mode 1): atomicMin of
// the triangle index among candidates whose key equals the minimum.
template <int MODE>
__global__ void __launch_bounds__(256) k_raster(TP P, const double *__restrict__ X, const double *__restrict__ Y,
                                                const int *__restrict__ L, uint64_t *__restrict__ tkey,
                                                uint64_t *__restrict__ ikey, uint64_t *__restrict__ tkey_rx,
                                                uint64_t *__restrict__ ikey_rx) {
    const int64_t cells_per = (int64_t)P.nmax * (P.nr - 1);
    const int64_t tot = cells_per * P.ne;
    const int64_t N = (int64_t)P.nx * P.ny;
    const double tol = -P.bary_tol;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int eb = (int)(idx / cells_per);
        const int64_t rem = idx - (int64_t)eb * cells_per;
        const int n = (int)(rem / (P.nr - 1));
        const int j = (int)(rem - (int64_t)n * (P.nr - 1));
        const int *Le = L + (size_t)eb * P.nr;
        if (n + 1 > Le[j] || n + 1 > Le[j + 1]) continue;
        const int64_t base = (int64_t)eb * (P.nmax + 1) * P.nr;
        uint64_t *tk = tkey + eb * N;
        uint64_t *ik = ikey + eb * N;
        uint64_t *tkr = tkey_rx + (int64_t)eb * P.m;
        uint64_t *ikr = ikey_rx + (int64_t)eb * P.m;
        for (int tri = 0; tri < 2; ++tri) {
            int64_t ka, kb, kc;
            int na, nb, nc;
            tri_nodes(base, n, j, P.nr, tri, ka, kb, kc, na, nb, nc);
            Tri t;
            if (!make_tri(X[ka], Y[ka], X[kb], Y[kb], X[kc], Y[kc], t)) continue;
            const double ta = (double)na * P.dtau, tb = (double)nb * P.dtau, tc = (double)nc * P.dtau;
            const uint64_t my = ((((uint64_t)n * P.nr) + j) << 1) | (uint64_t)tri;
            // pixel centres inside the closed bounding box
            double ilo = ceil((t.xmin - P.x0) / P.h), ihi = floor((t.xmax - P.x0) / P.h);
            double jlo = ceil((t.ymin - P.y0) / P.h), jhi = floor((t.ymax - P.y0) / P.h);
            if (ilo < 0.0) ilo = 0.0;
            if (jlo < 0.0) jlo = 0.0;
            if (ihi > (double)(P.nx - 1)) ihi = (double)(P.nx - 1);
            if (jhi > (double)(P.ny - 1)) jhi = (double)(P.ny - 1);
            if (ilo <= ihi && jlo <= jhi) {
                for (long jj = (long)jlo; jj <= (long)jhi; ++jj) {
                    for (long ii = (long)ilo; ii <= (long)ihi; ++ii) {
                        double la, lb, lc;
                        if (!bary(t, P.x0 + (double)ii * P.h, P.y0 + (double)jj * P.h, tol, la, lb, lc))
                            continue;
                        const double tv = la * ta + lb * tb + lc * tc;
                        const uint64_t key = order_key(tv);
                        const int64_t p = (int64_t)jj * P.nx + ii;
                        if (MODE == 0) {
                            atomicMin((unsigned long long *)&tk[p], (unsigned long long)key);
                        } else if (key == tk[p]) {
                            atomicMin((unsigned long long *)&ik[p], (unsigned long long)my);
                        }
                    }
                }
            }
            // ring elements
            int rlo, rhi;
            if (rx_range(P, t, rlo, rhi)) {
                for (int rr = rlo; rr <= rhi; ++rr) {
                    const int r = ((rr % P.m) + P.m) % P.m;
                    double px, py;
                    rx_pos(P, r, px, py);
                    if (px < t.xmin || px > t.xmax || py < t.ymin || py > t.ymax) continue;
                    double la, lb, lc;
                    if (!bary(t, px, py, tol, la, lb, lc)) continue;
                    const double tv = la * ta + lb * tb + lc * tc;
                    const uint64_t key = order_key(tv);
                    if (MODE == 0) {
                        atomicMin((unsigned long long *)&tkr[r], (unsigned long long)key);
                    } else if (key == tkr[r]) {
                        atomicMin((unsigned long long *)&ikr[r], (unsigned long long)my);
                    }
                }
            }
        }
    }
}

// Pass 3: every point recomputes its winning triangle's interpolation and
// writes T (in place of the key), a and B.  Points are pixels (RX = false)
// or ring elements (RX = true).
template <bool RX>
__global__ void k_raster_write(TP P, const double *__restrict__ X, const double *__restrict__ Y,
                               const double *__restrict__ Bn, const double *__restrict__ AMP,
                               uint64_t *__restrict__ tkey, const uint64_t *__restrict__ ikey,
                               float *__restrict__ amp_out, float *__restrict__ att_out) {
    const int64_t npts = RX ? (int64_t)P.m : (int64_t)P.nx * P.ny;
    const int64_t tot = npts * P.ne;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int eb = (int)(idx / npts);
        const int64_t p = idx - (int64_t)eb * npts;
        const uint64_t key = tkey[idx];
        double *Tout = reinterpret_cast<double *>(tkey);
        if (key == ~0ull) {
            Tout[idx] = __longlong_as_double(0x7ff8000000000000ll);
            amp_out[idx] = 0.0f;
            att_out[idx] = 0.0f;
            continue;
        }
        const uint64_t w = ikey[idx];
        const int tri = (int)(w & 1ull);
        const int64_t cell = (int64_t)(w >> 1);
        const int64_t n64 = cell / P.nr;
        const int j = (int)(cell - n64 * P.nr);
        if (w == ~0ull || n64 >= P.nmax || j >= P.nr - 1) {  // no winner recorded: uncovered
            Tout[idx] = __longlong_as_double(0x7ff8000000000000ll);
            amp_out[idx] = 0.0f;
            att_out[idx] = 0.0f;
            continue;
        }
        const int n = (int)n64;
        const int64_t base = (int64_t)eb * (P.nmax + 1) * P.nr;
        int64_t ka, kb, kc;
        int na, nb, nc;
        tri_nodes(base, n, j, P.nr, tri, ka, kb, kc, na, nb, nc);
        Tri t;
        make_tri(X[ka], Y[ka], X[kb], Y[kb], X[kc], Y[kc], t);
        double px, py;
        if (RX) {
            rx_pos(P, (int)p, px, py);
        } else {
            const int64_t jj = p / P.nx, ii = p - jj * P.nx;
            px = P.x0 + (double)ii * P.h;
            py = P.y0 + (double)jj * P.h;
        }
        double la, lb, lc;
        bary(t, px, py, -P.bary_tol, la, lb, lc);
        const double ta = (double)na * P.dtau, tb = (double)nb * P.dtau, tc = (double)nc * P.dtau;
        Tout[idx] = la * ta + lb * tb + lc * tc;
        amp_out[idx] = (float)(la * AMP[ka] + lb * AMP[kb] + lc * AMP[kc]);
        att_out[idx] = (float)(la * Bn[ka] + lb * Bn[kb] + lc * Bn[kc]);
    }
}

struct TraceWs {
    double2 *sa;
    double *X, *Y, *Bn, *AMP;
    int *L;
    uint64_t *ikey, *ikey_rx;
};

size_t per_emitter_bytes(const rb_geometry *g, const rb_trace_opts *t) {
    const size_t nodes = (size_t)(trace_nmax(t) + 1) * t->n_rays;
    return nodes * 4 * sizeof(double) + (size_t)t->n_rays * sizeof(int) +
           (size_t)g->nx * g->ny * sizeof(uint64_t) + (size_t)g->m * sizeof(uint64_t) + 8 * 256;
}

TraceWs carve_trace(Carver &c, const rb_geometry *g, const rb_trace_opts *t, int batch) {
    TraceWs w;
    const size_t N = (size_t)g->nx * g->ny;
    const size_t nodes = (size_t)(trace_nmax(t) + 1) * t->n_rays * batch;
    w.sa = c.take<double2>(N);
    w.X = c.take<double>(nodes);
    w.Y = c.take<double>(nodes);
    w.Bn = c.take<double>(nodes);
    w.AMP = c.take<double>(nodes);
    w.L = c.take<int>((size_t)t->n_rays * batch);
    w.ikey = c.take<uint64_t>(N * batch);
    w.ikey_rx = c.take<uint64_t>((size_t)g->m * batch);
    return w;
}

}  // namespace

size_t trace_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int batch) {
    if (check_trace(g, t) != RB_OK) return 0;
    if (batch <= 0 || batch > g->m) batch = g->m;
    Carver c(nullptr, 0);
    carve_trace(c, g, t, batch);
    return c.used + 256;
}

// Traces all emitters into `out`, in batches that fit the workspace.
rb_status trace_rays_impl(const rb_geometry *g, const rb_trace_opts *t, const double *slowness,
                          const double *alpha0, const rb_tables *out, void *ws, size_t ws_bytes,
                          hipStream_t st) {
    const int64_t N = (int64_t)g->nx * g->ny;
    // how many emitters fit
    Carver probe(nullptr, 0);
    carve_trace(probe, g, t, 1);
    const size_t one = probe.used + 256;
    if (ws_bytes < one) {
        set_error("trace workspace too small: need >= %zu bytes, got %zu", one, ws_bytes);
        return RB_ENOMEM;
    }
    int batch = (int)std::min<size_t>((size_t)g->m, 1 + (ws_bytes - one) / per_emitter_bytes(g, t));
    while (batch > 1) {
        Carver c2(nullptr, 0);
        carve_trace(c2, g, t, batch);
        if (c2.used + 256 <= ws_bytes) break;
        --batch;
    }
    char *base = reinterpret_cast<char *>(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    Carver c(base, ws_bytes - (size_t)(base - (char *)ws));
    TraceWs w = carve_trace(c, g, t, batch);

    TP P;
    P.nx = g->nx; P.ny = g->ny; P.h = g->h; P.x0 = g->x0; P.y0 = g->y0;
    P.m = g->m; P.R = g->ring_radius; P.s_bg = 1.0 / g->c_background;
    P.nr = t->n_rays; P.dtau = t->dtau; P.nmax = (int)trace_nmax(t);
    const double r_die = g->ring_radius + 2.0 * g->h;
    P.rdie2 = r_die * r_die;
    P.j_min = t->j_min > 0.0 ? t->j_min : 0.25 * g->h;
    P.bary_tol = 1e-12;
    const double dpsi = M_PI / (double)t->n_rays;
    P.two_sin_full = 2.0 * std::sin(dpsi);
    P.two_sin_half = 2.0 * std::sin(0.5 * dpsi);

    k_pack<<<blocks_for(N, 256), 256, 0, st>>>(slowness, alpha0, N, w.sa);
    RB_LAUNCHED();
    for (int e0 = 0; e0 < g->m; e0 += batch) {
        P.e0 = e0;
        P.ne = std::min(batch, g->m - e0);
        uint64_t *tkey = reinterpret_cast<uint64_t *>(out->T + (int64_t)e0 * N);
        uint64_t *tkey_rx = reinterpret_cast<uint64_t *>(out->T_rx + (int64_t)e0 * g->m);
        RB_TRY(fill_u64(tkey, ~0ull, (int64_t)P.ne * N, st));
        RB_TRY(fill_u64(w.ikey, ~0ull, (int64_t)P.ne * N, st));
        RB_TRY(fill_u64(tkey_rx, ~0ull, (int64_t)P.ne * g->m, st));
        RB_TRY(fill_u64(w.ikey_rx, ~0ull, (int64_t)P.ne * g->m, st));
        dim3 gt(blocks_for(P.nr, 128), P.ne);
        k_trace<<<gt, 128, 0, st>>>(P, w.sa, w.X, w.Y, w.Bn, w.L);
        RB_LAUNCHED();
        const int64_t nodes = (int64_t)(P.nmax + 1) * P.nr * P.ne;
        unsigned bs = (unsigned)std::min<int64_t>(blocks_for(nodes, 256), 1 << 20);
        k_spread<<<bs, 256, 0, st>>>(P, w.sa, w.X, w.Y, w.L, w.AMP);
        RB_LAUNCHED();
        const int64_t cells = (int64_t)P.nmax * (P.nr - 1) * P.ne;
        unsigned bc = (unsigned)std::min<int64_t>(blocks_for(cells, 256), 1 << 20);
        k_raster<0><<<bc, 256, 0, st>>>(P, w.X, w.Y, w.L, tkey, w.ikey, tkey_rx, w.ikey_rx);
        RB_LAUNCHED();
        k_raster<1><<<bc, 256, 0, st>>>(P, w.X, w.Y, w.L, tkey, w.ikey, tkey_rx, w.ikey_rx);
        RB_LAUNCHED();
        const int64_t npx = N * P.ne;
        k_raster_write<false><<<(unsigned)std::min<int64_t>(blocks_for(npx, 256), 1 << 20), 256, 0, st>>>(
            P, w.X, w.Y, w.Bn, w.AMP, tkey, w.ikey, out->amp + (int64_t)e0 * N, out->att + (int64_t)e0 * N);
        RB_LAUNCHED();
        const int64_t nrx = (int64_t)g->m * P.ne;
        k_raster_write<true><<<blocks_for(nrx, 256), 256, 0, st>>>(
            P, w.X, w.Y, w.Bn, w.AMP, tkey_rx, w.ikey_rx, out->amp_rx + (int64_t)e0 * g->m,
            out->att_rx + (int64_t)e0 * g->m);
        RB_LAUNCHED();
    }
    return RB_OK;
}

rb_status check_tables(const rb_tables *t) {
    RB_CHECK_ARG(t != nullptr, "tables are NULL");
    RB_CHECK_ARG(t->T && t->amp && t->att && t->T_rx && t->amp_rx && t->att_rx,
                 "all six table pointers are required");
    return RB_OK;
}

}  // namespace rb

extern "C" {

size_t rb_trace_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int32_t emitter_batch) {
    return rb::trace_workspace_bytes(g, t, emitter_batch);
}

rb_status rb_trace_rays(const rb_geometry *g, const rb_trace_opts *t, const double *slowness,
                        const double *alpha0, const rb_tables *out, void *ws, size_t ws_bytes,
                        void *stream) {
    rb::clear_error();
    RB_TRY(rb::check_trace(g, t));
    RB_TRY(rb::check_tables(out));
    RB_CHECK_ARG(slowness != nullptr, "slowness is NULL");
    RB_CHECK_ARG(ws != nullptr, "workspace is NULL");
    return rb::trace_rays_impl(g, t, slowness, alpha0, out, ws, ws_bytes, rb::as_stream(stream));
}

}  // extern "C"
