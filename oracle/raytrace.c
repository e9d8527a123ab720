/*
 * FP64 reference oracle: ray tracing, spreading amplitude and ray-to-grid
 * interpolation for the ray-Born Green's functions.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU definition that the GPU library is checked against.  Nothing in the
 * product path may link or call it.  Built with gcc -O2 -ffp-contract=off so
 * every operation below is one IEEE double rounding, in the written order.
 *
 * What it computes (paper, "Forward Problem" section):
 *   - the Green's function is approximated as A exp(i[phi + pi/4]) (Eq. 4)
 *     with phi = omega*T and A = A_geom * A_abs (Eq. 5);
 *   - T solves the Eikonal equation |grad T| = s (Eq. 6 divided by omega^2),
 *     integrated along rays with travel time tau as the ray parameter:
 *         dx/dtau = p / s^2,   dp/dtau = grad(s) / s,
 *     so that the travel time at node n is exactly n*dtau;
 *   - absorption accumulates along the ray: dB/dtau = alpha0(x) / s(x),
 *     i.e. B = integral of alpha0 over arclength;
 *   - A_geom follows from the Transport equation (Eq. 7): the energy flux
 *     A^2 |grad phi| J through a ray tube of width J dpsi is constant, which,
 *     normalised to the 2-D point-source far field, gives
 *         A_geom = sqrt(c(x) / (8 pi omega J)),  J = |dx/dpsi| at fixed tau;
 *     the omega^(-1/2) factor is applied when G is formed, this file
 *     stores a = sqrt(c / (8 pi max(J, j_min))).
 * The ray-to-grid step (the Discussion's carrying of the ray parameters back
 * onto the grid) is done on the wavefront mesh: cell (j, n) spans rays j, j+1 and nodes
 * n, n+1 and is split into the triangles (P[n][j], P[n][j+1], P[n+1][j+1])
 * and (P[n][j], P[n+1][j+1], P[n+1][j]); a point inside a triangle takes
 * the barycentric interpolation of T, a and B; over all covering triangles
 * the first arrival wins: the candidate with the smallest interpolated
 * travel time T = la T_a + lb T_b + lc T_c, computed in FP64 and compared
 * exactly; equal values go to the first triangle in (n, j, triangle) order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny;
    double h, x0, y0;
    int32_t m;
    double R;       /* ring radius */
    double s_bg;    /* slowness outside the grid */
    int32_t n_rays;
    double dtau;    /* travel-time step */
    int32_t nmax;   /* maximum number of steps */
    double r_die;   /* a ray ends at the first node with |x| > r_die */
    double j_min;   /* floor on the spreading J */
    double bary_tol;
} orc_params;

/* value of a grid field at integer pixel (i, j); `out` outside the grid */
static double at(const double *f, const orc_params *P, long i, long j, double out)
{
    if (i < 0 || j < 0 || i >= P->nx || j >= P->ny) return out;
    return f[(size_t)j * (size_t)P->nx + (size_t)i];
}

/* Bilinear interpolation between pixel centres, and the exact gradient of
 * that bilinear patch.  The field takes `out` at pixels outside the grid. */
static void bilinear(const double *f, double out, const orc_params *P,
                     double x, double y, double *val, double *gx, double *gy)
{
    double u = (x - P->x0) / P->h;
    double v = (y - P->y0) / P->h;
    double fi = floor(u), fj = floor(v);
    if (!(fi >= -1.0 && fi <= (double)P->nx && fj >= -1.0 && fj <= (double)P->ny)) {
        *val = out; *gx = 0.0; *gy = 0.0;   /* all four corners outside */
        return;
    }
    long i = (long)fi, j = (long)fj;
    double fu = u - fi, fv = v - fj;
    double s00 = at(f, P, i, j, out),     s10 = at(f, P, i + 1, j, out);
    double s01 = at(f, P, i, j + 1, out), s11 = at(f, P, i + 1, j + 1, out);
    double dx0 = s10 - s00, dx1 = s11 - s01;
    double s0 = s00 + fu * dx0;
    double s1 = s01 + fu * dx1;
    *val = s0 + fv * (s1 - s0);
    *gx = (dx0 + fv * (dx1 - dx0)) / P->h;
    *gy = (s1 - s0) / P->h;
}

/* right-hand side of the ray equations, state = (x, y, px, py, B) */
static void rhs(const orc_params *P, const double *s, const double *alpha,
                const double st[5], double d[5])
{
    double sv, sx, sy, av = 0.0, ax, ay;
    bilinear(s, P->s_bg, P, st[0], st[1], &sv, &sx, &sy);
    if (alpha) bilinear(alpha, 0.0, P, st[0], st[1], &av, &ax, &ay);
    double s2 = sv * sv;
    d[0] = st[2] / s2;
    d[1] = st[3] / s2;
    d[2] = sx / sv;
    d[3] = sy / sv;
    d[4] = av / sv;
}

/* classic four-stage Runge-Kutta step of length dt */
static void rk4(const orc_params *P, const double *s, const double *alpha,
                double st[5], double dt)
{
    double k1[5], k2[5], k3[5], k4[5], t[5];
    double hdt = 0.5 * dt, sixth = dt / 6.0;
    int q;
    rhs(P, s, alpha, st, k1);
    for (q = 0; q < 5; ++q) t[q] = st[q] + hdt * k1[q];
    rhs(P, s, alpha, t, k2);
    for (q = 0; q < 5; ++q) t[q] = st[q] + hdt * k2[q];
    rhs(P, s, alpha, t, k3);
    for (q = 0; q < 5; ++q) t[q] = st[q] + dt * k3[q];
    rhs(P, s, alpha, t, k4);
    for (q = 0; q < 5; ++q)
        st[q] = st[q] + sixth * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
}

/*
 * Trace the fan of emitter e.  Output arrays are [(nmax+1) * n_rays], node
 * (n, j) at n*n_rays + j: position X, Y, slowness vector PX, PY, absorption
 * integral Bn and amplitude factor AMP.  L[j] is the last node of ray j.
 * The fan covers the inward half-plane: psi_j = theta_e + pi +
 * (j + 1/2 - n_rays/2) * pi/n_rays, the tangent directions excluded.
 */
int orc_trace_fan(const orc_params *P, const double *s, const double *alpha, int e,
                  double *X, double *Y, double *PX, double *PY, double *Bn,
                  double *AMP, int32_t *L)
{
    const int nr = P->n_rays;
    const double theta = 2.0 * M_PI * (double)e / (double)P->m;
    const double xe = P->R * cos(theta), ye = P->R * sin(theta);
    const double dpsi = M_PI / (double)nr;
    const double rdie2 = P->r_die * P->r_die;
    double se, gx, gy;
    bilinear(s, P->s_bg, P, xe, ye, &se, &gx, &gy);
    for (int j = 0; j < nr; ++j) {
        double psi = theta + M_PI + ((double)j + 0.5 - 0.5 * (double)nr) * dpsi;
        double st[5] = {xe, ye, se * cos(psi), se * sin(psi), 0.0};
        X[j] = st[0]; Y[j] = st[1]; PX[j] = st[2]; PY[j] = st[3]; Bn[j] = 0.0;
        int last = P->nmax;
        for (int n = 0; n < P->nmax; ++n) {
            rk4(P, s, alpha, st, P->dtau);
            size_t k = (size_t)(n + 1) * nr + j;
            X[k] = st[0]; Y[k] = st[1]; PX[k] = st[2]; PY[k] = st[3]; Bn[k] = st[4];
            if (st[0] * st[0] + st[1] * st[1] > rdie2) { last = n + 1; break; }
        }
        L[j] = last;
    }
    /* spreading from the neighbouring rays at equal travel time */
    const double two_sin_full = 2.0 * sin(dpsi);
    const double two_sin_half = 2.0 * sin(0.5 * dpsi);
    const double eight_pi = 8.0 * M_PI;
    int nmax_alive = 0;
    for (int j = 0; j < nr; ++j) if (L[j] > nmax_alive) nmax_alive = L[j];
    for (int n = 0; n <= nmax_alive; ++n) {
        for (int j = 0; j < nr; ++j) {
            if (n > L[j]) continue;
            size_t k = (size_t)n * nr + j;
            int lo = (j > 0 && n <= L[j - 1]);
            int hi = (j + 1 < nr && n <= L[j + 1]);
            double Jv = 0.0, dx, dy;
            if (lo && hi) {
                dx = X[k + 1] - X[k - 1]; dy = Y[k + 1] - Y[k - 1];
                Jv = sqrt(dx * dx + dy * dy) / two_sin_full;
            } else if (hi) {
                dx = X[k + 1] - X[k]; dy = Y[k + 1] - Y[k];
                Jv = sqrt(dx * dx + dy * dy) / two_sin_half;
            } else if (lo) {
                dx = X[k] - X[k - 1]; dy = Y[k] - Y[k - 1];
                Jv = sqrt(dx * dx + dy * dy) / two_sin_half;
            }
            if (Jv < P->j_min) Jv = P->j_min;
            double sv;
            bilinear(s, P->s_bg, P, X[k], Y[k], &sv, &gx, &gy);
            AMP[k] = sqrt((1.0 / sv) / (eight_pi * Jv));
        }
    }
    return 0;
}

/* One triangle: evaluate at the candidate points inside its closed bounding
 * box; keep the smallest interpolated T per point in Q (strict <, so the
 * triangles visited earlier keep exact ties). */
typedef struct { double x, y, t, a, b; } vtx;

static void raster_grid(const orc_params *P, const vtx *A, const vtx *B, const vtx *C,
                        double *Q, double *T, double *Am, double *Bt)
{
    double e1x = B->x - A->x, e1y = B->y - A->y;
    double e2x = C->x - A->x, e2y = C->y - A->y;
    double det = e1x * e2y - e1y * e2x;
    if (det == 0.0) return;
    double xmin = fmin(A->x, fmin(B->x, C->x)), xmax = fmax(A->x, fmax(B->x, C->x));
    double ymin = fmin(A->y, fmin(B->y, C->y)), ymax = fmax(A->y, fmax(B->y, C->y));
    double ilo = ceil((xmin - P->x0) / P->h), ihi = floor((xmax - P->x0) / P->h);
    double jlo = ceil((ymin - P->y0) / P->h), jhi = floor((ymax - P->y0) / P->h);
    if (ilo < 0.0) ilo = 0.0;
    if (jlo < 0.0) jlo = 0.0;
    if (ihi > (double)(P->nx - 1)) ihi = (double)(P->nx - 1);
    if (jhi > (double)(P->ny - 1)) jhi = (double)(P->ny - 1);
    if (ilo > ihi || jlo > jhi) return;
    const double tol = -P->bary_tol;
    for (long jj = (long)jlo; jj <= (long)jhi; ++jj) {
        for (long ii = (long)ilo; ii <= (long)ihi; ++ii) {
            double qx = (P->x0 + (double)ii * P->h) - A->x;
            double qy = (P->y0 + (double)jj * P->h) - A->y;
            double lb = (qx * e2y - qy * e2x) / det;
            double lc = (e1x * qy - e1y * qx) / det;
            double la = (1.0 - lb) - lc;
            if (la < tol || lb < tol || lc < tol) continue;
            double t = la * A->t + lb * B->t + lc * C->t;
            size_t p = (size_t)jj * (size_t)P->nx + (size_t)ii;
            if (t < Q[p]) {
                Q[p] = t;
                T[p] = t;
                Am[p] = la * A->a + lb * B->a + lc * C->a;
                Bt[p] = la * A->b + lb * B->b + lc * C->b;
            }
        }
    }
}

static void raster_points(const orc_params *P, const vtx *A, const vtx *B, const vtx *C,
                          int npts, const double *px, const double *py,
                          double *Q, double *T, double *Am, double *Bt,
                          int64_t tri_index, int64_t *Wi, double *Wl)
{
    double e1x = B->x - A->x, e1y = B->y - A->y;
    double e2x = C->x - A->x, e2y = C->y - A->y;
    double det = e1x * e2y - e1y * e2x;
    if (det == 0.0) return;
    double xmin = fmin(A->x, fmin(B->x, C->x)), xmax = fmax(A->x, fmax(B->x, C->x));
    double ymin = fmin(A->y, fmin(B->y, C->y)), ymax = fmax(A->y, fmax(B->y, C->y));
    /* the points lie on the ring |x| = R: skip boxes that miss it (with slack) */
    double dxm = xmin > 0.0 ? xmin : (xmax < 0.0 ? -xmax : 0.0);
    double dym = ymin > 0.0 ? ymin : (ymax < 0.0 ? -ymax : 0.0);
    double dmin = sqrt(dxm * dxm + dym * dym);
    double dmax = sqrt(fmax(xmin * xmin, xmax * xmax) + fmax(ymin * ymin, ymax * ymax));
    if (dmin > P->R * (1.0 + 1e-9) || dmax < P->R * (1.0 - 1e-9)) return;
    const double tol = -P->bary_tol;
    for (int r = 0; r < npts; ++r) {
        if (px[r] < xmin || px[r] > xmax || py[r] < ymin || py[r] > ymax) continue;
        double qx = px[r] - A->x, qy = py[r] - A->y;
        double lb = (qx * e2y - qy * e2x) / det;
        double lc = (e1x * qy - e1y * qx) / det;
        double la = (1.0 - lb) - lc;
        if (la < tol || lb < tol || lc < tol) continue;
        double t = la * A->t + lb * B->t + lc * C->t;
        if (t < Q[r]) {
            Q[r] = t;
            T[r] = t;
            Am[r] = la * A->a + lb * B->a + lc * C->a;
            Bt[r] = la * A->b + lb * B->b + lc * C->b;
            if (Wi) {   /* the winning triangle and the point's barycentrics */
                Wi[r] = tri_index;
                Wl[3 * r] = la; Wl[3 * r + 1] = lb; Wl[3 * r + 2] = lc;
            }
        }
    }
}

/*
 * Ray-to-grid tables for emitters [e0, e1): T, amplitude factor a and
 * absorption integral B at every pixel centre ([e1-e0][ny*nx]) and at every
 * ring element ([e1-e0][m]).  Uncovered entries hold NaN (T) and 0 (a, B).
 * Emitters are independent; with OpenMP each thread traces its own fans.
 */
int orc_tables(const orc_params *P, const double *s, const double *alpha, int e0, int e1,
               double *T, double *Am, double *Bt, double *Trx, double *Arx, double *Brx)
{
    const size_t N = (size_t)P->nx * (size_t)P->ny;
    const int nr = P->n_rays, m = P->m;
    double *px = (double *)malloc(sizeof(double) * m);
    double *py = (double *)malloc(sizeof(double) * m);
    for (int r = 0; r < m; ++r) {
        double th = 2.0 * M_PI * (double)r / (double)m;
        px[r] = P->R * cos(th); py[r] = P->R * sin(th);
    }
    int status = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int e = e0; e < e1; ++e) {
        size_t nn = (size_t)(P->nmax + 1) * nr;
        double *X = (double *)malloc(sizeof(double) * nn * 6);
        int32_t *L = (int32_t *)malloc(sizeof(int32_t) * nr);
        double *Q = (double *)malloc(sizeof(double) * (N + (size_t)m));
        if (!X || !L || !Q) { status = -2; free(X); free(L); free(Q); continue; }
        double *Qr = Q + N;
        double *Y = X + nn, *PX = Y + nn, *PY = PX + nn, *Bn = PY + nn, *AMP = Bn + nn;
        orc_trace_fan(P, s, alpha, e, X, Y, PX, PY, Bn, AMP, L);
        double *Te = T + (size_t)(e - e0) * N, *Ae = Am + (size_t)(e - e0) * N;
        double *Be = Bt + (size_t)(e - e0) * N;
        double *Tr = Trx + (size_t)(e - e0) * m, *Ar = Arx + (size_t)(e - e0) * m;
        double *Br = Brx + (size_t)(e - e0) * m;
        for (size_t p = 0; p < N; ++p) { Q[p] = INFINITY; Te[p] = NAN; Ae[p] = 0.0; Be[p] = 0.0; }
        for (int r = 0; r < m; ++r) { Qr[r] = INFINITY; Tr[r] = NAN; Ar[r] = 0.0; Br[r] = 0.0; }
        for (int n = 0; n < P->nmax; ++n) {
            for (int j = 0; j + 1 < nr; ++j) {
                if (n + 1 > L[j] || n + 1 > L[j + 1]) continue;
                size_t k00 = (size_t)n * nr + j, k10 = k00 + 1;
                size_t k01 = k00 + nr, k11 = k01 + 1;
                double t0 = (double)n * P->dtau, t1 = (double)(n + 1) * P->dtau;
                vtx p00 = {X[k00], Y[k00], t0, AMP[k00], Bn[k00]};
                vtx p10 = {X[k10], Y[k10], t0, AMP[k10], Bn[k10]};
                vtx p11 = {X[k11], Y[k11], t1, AMP[k11], Bn[k11]};
                vtx p01 = {X[k01], Y[k01], t1, AMP[k01], Bn[k01]};
                raster_grid(P, &p00, &p10, &p11, Q, Te, Ae, Be);
                raster_points(P, &p00, &p10, &p11, m, px, py, Qr, Tr, Ar, Br, 0, NULL, NULL);
                raster_grid(P, &p00, &p11, &p01, Q, Te, Ae, Be);
                raster_points(P, &p00, &p11, &p01, m, px, py, Qr, Tr, Ar, Br, 0, NULL, NULL);
            }
        }
        free(X); free(L); free(Q);
    }
    free(px); free(py);
    return status;
}

/*
 * First arrivals of emitter e's fan at the ring elements, with the winning
 * triangle: for every element r, T[r] (NaN if uncovered), the triangle
 * index W[r] = 2 (n n_rays + j) + t (t = 0: (P[n][j], P[n][j+1],
 * P[n+1][j+1]); t = 1: (P[n][j], P[n+1][j+1], P[n+1][j]); -1 if uncovered)
 * and the element's barycentrics (la, lb, lc) in it, in the order of those
 * vertices.  Same rule and arithmetic as orc_tables.  The fan's nodes are
 * returned in X, Y ([(nmax+1) n_rays]) and L ([n_rays]) as by orc_trace_fan.
 */
int orc_rx_links(const orc_params *P, const double *s, const double *alpha, int e,
                 double *X, double *Y, int32_t *L, double *T, int64_t *W, double *Wl)
{
    const int nr = P->n_rays, m = P->m;
    size_t nn = (size_t)(P->nmax + 1) * nr;
    double *buf = (double *)malloc(sizeof(double) * nn * 4 + sizeof(double) * 4 * m);
    double *Qr = (double *)malloc(sizeof(double) * m);
    if (!buf || !Qr) { free(buf); free(Qr); return -2; }
    double *PX = buf, *PY = PX + nn, *Bn = PY + nn, *AMP = Bn + nn;
    double *px = AMP + nn, *py = px + m, *Ar = py + m, *Br = Ar + m;
    for (int r = 0; r < m; ++r) {
        double th = 2.0 * M_PI * (double)r / (double)m;
        px[r] = P->R * cos(th); py[r] = P->R * sin(th);
        Qr[r] = INFINITY; T[r] = NAN; W[r] = -1;
        Wl[3 * r] = Wl[3 * r + 1] = Wl[3 * r + 2] = 0.0;
    }
    orc_trace_fan(P, s, alpha, e, X, Y, PX, PY, Bn, AMP, L);
    for (int n = 0; n < P->nmax; ++n) {
        for (int j = 0; j + 1 < nr; ++j) {
            if (n + 1 > L[j] || n + 1 > L[j + 1]) continue;
            size_t k00 = (size_t)n * nr + j, k10 = k00 + 1;
            size_t k01 = k00 + nr, k11 = k01 + 1;
            double t0 = (double)n * P->dtau, t1 = (double)(n + 1) * P->dtau;
            vtx p00 = {X[k00], Y[k00], t0, AMP[k00], Bn[k00]};
            vtx p10 = {X[k10], Y[k10], t0, AMP[k10], Bn[k10]};
            vtx p11 = {X[k11], Y[k11], t1, AMP[k11], Bn[k11]};
            vtx p01 = {X[k01], Y[k01], t1, AMP[k01], Bn[k01]};
            const int64_t cell = (int64_t)n * nr + j;
            raster_points(P, &p00, &p10, &p11, m, px, py, Qr, T, Ar, Br, 2 * cell, W, Wl);
            raster_points(P, &p00, &p11, &p01, m, px, py, Qr, T, Ar, Br, 2 * cell + 1, W, Wl);
        }
    }
    free(buf); free(Qr);
    return 0;
}

/* Bilinear slowness and gradient at arbitrary points (used by tests). */
void orc_bilinear(const orc_params *P, const double *f, double out, int npts,
                  const double *x, const double *y, double *val, double *gx, double *gy)
{
    for (int k = 0; k < npts; ++k) bilinear(f, out, P, x[k], y[k], &val[k], &gx[k], &gy[k]);
}
