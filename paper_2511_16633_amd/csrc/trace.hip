// Ray tracing and ray-to-grid tables.
//
// Model (paper, Forward Problem section): the travel time T solves the
// Eikonal equation (Eq. 6), integrated along rays with T itself as the ray
// parameter; the amplitude follows from the Transport equation (Eq. 7) via
// the ray-tube width J from neighbouring rays; absorption accumulates along
// each ray (Eq. 5).  The tables are formed on the wavefront mesh (the
// Discussion carries the ray parameters back onto the grid) by first-arrival
// barycentric interpolation.
//
// GPU design:
//  * one lane per ray, classic RK4 in FP64; the slowness and absorption maps
//    are packed into one 16-byte (s, alpha0) record per pixel so a bilinear
//    corner is one load, served from L2/MALL (a 480x480 map is 3.7 MB);
//  * wavefront nodes are stored [emitter][step][ray] so the lanes of a wave
//    write consecutive addresses at every step (24 bytes a node);
//  * first arrival without floating-point atomics: the tracing waves list
//    the mesh cells whose bounding box holds a pixel centre or straddles the
//    ring as the cells close; the raster passes take one 64-bit atomicMin per
//    candidate on the arrival key (fixed-point step index above the
//    triangle index), and the write pass decodes each point's winner and
//    recomputes its barycentrics.  The result is independent of scheduling;
//  * the bent-ray ToF starting model reads each pair's linking path from the
//    arrival key at the receiving element (end of this file).
#include <climits>
#include <cmath>
#include <type_traits>

#include "common.h"
#include "green.h"

namespace rb {
namespace {

struct TP {
    int nx, ny;
    double h, x0, y0;
    double inv_h;      // 1 / h
    int m;
    double R, s_bg;
    int nr;            // rays per emitter
    double dtau;
    int nmax;
    double rdie2;      // (R + 2h)^2
    double j_min;
    double bary_tol;
    double inv_chord_full, inv_chord_half;   // 1 / (2 sin dpsi), 1 / (2 sin (dpsi / 2))
    double ring2_lo, ring2_hi;  // (R (1 -+ 2e-9))^2: conservative ring test on squares
    int e0, ne;        // emitter batch
    int idx_bits;      // bits of the triangle index in an arrival key
    double qscale;     // 2^F: fixed-point scale of the step index in an arrival key
};

// Bilinear slowness s with its exact patch gradient, and bilinear alpha0.
// `sa` is the (s, alpha0) grid padded with two rings of water cells, row
// stride nx + 4.  Every cell that touches the grid has its four corners in
// memory, and a point farther out is evaluated in a clamped cell of the
// outer ring, whose four corners are all water: the value is exactly s_bg
// with zero gradient and no absorption, with no test or branch.
__device__ __forceinline__ void field(const double2 *__restrict__ sa, const TP &P, double x, double y,
                                      double &s, double &gx, double &gy, double &a) {
#pragma clang fp contract(fast)
    double u = (x - P.x0) * P.inv_h;
    double v = (y - P.y0) * P.inv_h;
    double fi = floor(u), fj = floor(v);
    // cells -2 .. n (padded 0 .. n + 2, corners up to n + 3)
    const int i = (int)fmin(fmax(fi, -2.0), (double)P.nx) + 2;
    const int j = (int)fmin(fmax(fj, -2.0), (double)P.ny) + 2;
    double fu = u - fi, fv = v - fj;
    const int ld = P.nx + 4;
    const double2 *q = sa + (j * ld + i);
    const double2 c00 = q[0], c10 = q[1], c01 = q[ld], c11 = q[ld + 1];
    double dx0 = c10.x - c00.x, dx1 = c11.x - c01.x;
    double s0 = c00.x + fu * dx0;
    double s1 = c01.x + fu * dx1;
    s = s0 + fv * (s1 - s0);
    gx = (dx0 + fv * (dx1 - dx0)) * P.inv_h;
    gy = (s1 - s0) * P.inv_h;
    double a0 = c00.y + fu * (c10.y - c00.y);
    double a1 = c01.y + fu * (c11.y - c01.y);
    a = a0 + fv * (a1 - a0);
}

// The same evaluation with the four corner records of the last cell kept in
// registers: a lane reloads them only when its point has left that cell.
// The four RK4 stages of a step lie within one step length (less than a
// cell), so most stages of most lanes reuse the corners, and the gathers -
// the tracer's bottleneck in the vector-memory path - shrink to the lanes
// that crossed a cell edge.  The values are those of field().
struct FieldCache {
    int i = -1, j = -1;   // padded cell whose corners are held (none yet)
    double2 c00, c10, c01, c11;
};

__device__ __forceinline__ void field_cached(const double2 *__restrict__ sa, const TP &P, double x, double y,
                                             FieldCache &fc, double &s, double &gx, double &gy, double &a) {
#pragma clang fp contract(fast)
    double u = (x - P.x0) * P.inv_h;
    double v = (y - P.y0) * P.inv_h;
    double fi = floor(u), fj = floor(v);
    const int i = (int)fmin(fmax(fi, -2.0), (double)P.nx) + 2;
    const int j = (int)fmin(fmax(fj, -2.0), (double)P.ny) + 2;
    double fu = u - fi, fv = v - fj;
    if (i != fc.i || j != fc.j) {
        const int ld = P.nx + 4;
        const double2 *q = sa + (j * ld + i);
        fc.c00 = q[0];
        fc.c10 = q[1];
        fc.c01 = q[ld];
        fc.c11 = q[ld + 1];
        fc.i = i;
        fc.j = j;
    }
    double dx0 = fc.c10.x - fc.c00.x, dx1 = fc.c11.x - fc.c01.x;
    double s0 = fc.c00.x + fu * dx0;
    double s1 = fc.c01.x + fu * dx1;
    s = s0 + fv * (s1 - s0);
    gx = (dx0 + fv * (dx1 - dx0)) * P.inv_h;
    gy = (s1 - s0) * P.inv_h;
    double a0 = fc.c00.y + fu * (fc.c10.y - fc.c00.y);
    double a1 = fc.c01.y + fu * (fc.c11.y - fc.c01.y);
    a = a0 + fv * (a1 - a0);
}

// 1/s from the hardware reciprocal refined by two Newton steps (to within
// an ulp of the correctly rounded quotient).
__device__ __forceinline__ double recip(double s) {
    double r = __builtin_amdgcn_rcp(s);
    r = r * (2.0 - s * r);
    r = r * (2.0 - s * r);
    return r;
}

__device__ __forceinline__ void rhs(const double2 *__restrict__ sa, const TP &P, const double st[5],
                                    FieldCache &fc, double d[5]) {
#pragma clang fp contract(fast)
    double s, gx, gy, a;
    field_cached(sa, P, st[0], st[1], fc, s, gx, gy, a);
    const double is = recip(s);
    const double is2 = is * is;
    d[0] = st[2] * is2;
    d[1] = st[3] * is2;
    d[2] = gx * is;
    d[3] = gy * is;
    d[4] = a * is;
}

__global__ void k_pack(int nx, int ny, double s_bg, const double *__restrict__ s, const double *__restrict__ alpha,
                       double2 *__restrict__ sa) {
    const int64_t np = (int64_t)(nx + 4) * (ny + 4);
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    const int jp = (int)(q / (nx + 4)), ip = (int)(q - (int64_t)jp * (nx + 4));
    const int i = ip - 2, j = jp - 2;
    if (i < 0 || j < 0 || i >= nx || j >= ny) {
        sa[q] = make_double2(s_bg, 0.0);
    } else {
        const int64_t p = (int64_t)j * nx + i;
        sa[q] = make_double2(s[p], alpha ? alpha[p] : 0.0);
    }
}

// Cell ids: (batch emitter << 31) | (step << 13) | ray.
__device__ __forceinline__ uint64_t cell_id(int eb, int n, int j) {
    return ((uint64_t)eb << 31) | ((uint64_t)n << 13) | (uint64_t)j;
}
__device__ __forceinline__ void cell_decode(uint64_t id, int &eb, int &n, int &j) {
    j = (int)(id & 8191u);
    n = (int)((id >> 13) & 262143u);
    eb = (int)(id >> 31);
}

// Rays of one emitter are traced a wave at a time in lockstep: lanes 1..62
// own rays j0 .. j0+61 and lanes 0 and 63 trace the neighbouring rays as a
// halo, so the ray-tube width J at every node of an owned ray comes from
// lane shuffles at equal travel time.  The slowness at a node is the first
// RK4 stage of the step that leaves it, so the amplitude factor
// a = sqrt(c / (8 pi max(J, j_min))) costs no extra field evaluation.
// Nodes are stored [eb][n][j]: positions as double pairs, (a, B) as float
// pairs (a is formed in FP32 and the tables store B in FP32).
//
// The same lockstep classifies the wavefront-mesh cells as they close: once
// node n of rays j and j + 1 exists, cell (n - 1, j) has its four corners in
// the registers of lanes j and j + 1 (two steps apart), so its bounding box
// is tested here and not in a pass that reads the nodes back.  A cell whose
// box holds a pixel centre goes to the pixel list, one whose box straddles
// the ring to the ring list (both tests conservative: each triangle's box
// lies inside its cell's).  Each wave appends to a private segment of each
// list (segment = (batch emitter, wave), capacity 62 nmax) with ballot
// prefixes, so there is no contended counter.
constexpr int kOwn = 62;
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf2 __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(256) k_trace(TP P, const double2 *__restrict__ sa, double2 *__restrict__ XY,
                                               float2 *__restrict__ AB, int *__restrict__ L, int64_t cap,
                                               uint64_t *__restrict__ list_px, uint64_t *__restrict__ list_rx,
                                               int *__restrict__ seg_px, int *__restrict__ seg_rx) {
    // the integration may fuse multiply-adds (one rounding instead of two)
#pragma clang fp contract(fast)
    const int lane = threadIdx.x & 63;
    const int nw = (P.nr + kOwn - 1) / kOwn;   // waves per emitter
    const int wv = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int eb = blockIdx.y;
    if (wv >= nw || eb >= P.ne) return;  // wave-uniform
    const int j = wv * kOwn + lane - 1;
    const bool valid = j >= 0 && j < P.nr;
    const bool own = valid && lane >= 1 && lane <= kOwn;
    const int e = P.e0 + eb;
    const double theta = 2.0 * M_PI * (double)e / (double)P.m;
    const double xe = P.R * cos(theta), ye = P.R * sin(theta);
    const double dpsi = M_PI / (double)P.nr;
    double se, gx, gy, av;
    field(sa, P, xe, ye, se, gx, gy, av);
    const double psi = theta + M_PI + ((double)j + 0.5 - 0.5 * (double)P.nr) * dpsi;
    double st[5] = {xe, ye, se * cos(psi), se * sin(psi), 0.0};
    const size_t base = (size_t)eb * (size_t)(P.nmax + 1) * P.nr + (valid ? j : 0);
    const double dt = P.dtau, hdt = 0.5 * dt, sixth = dt / 6.0;
    const double eight_pi = 8.0 * M_PI;
    const int64_t seg = (int64_t)eb * nw + wv;
    uint64_t *lp = list_px + seg * cap;
    uint64_t *lr = list_rx + seg * cap;
    const uint64_t below = (1ull << lane) - 1ull;
    const bool has_right = own && j + 1 < P.nr;   // cells (., j) exist
    int cp = 0, cr = 0;                          // wave-uniform list counts
    double xp = 0.0, yp = 0.0;                   // node n - 1 of this ray
    bool alive = valid;   // alive at the current node n
    FieldCache fc;
    bool last = false;    // the current node is the ray's last
    for (int n = 0; n <= P.nmax; ++n) {
        if (!__any(alive)) break;
        // field at the node (first RK4 stage of the next step)
        double s0 = 1.0, g0x = 0.0, g0y = 0.0, a0 = 0.0;
        if (alive) field_cached(sa, P, st[0], st[1], fc, s0, g0x, g0y, a0);
        // neighbours at equal travel time
        const double xl = __shfl_up(st[0], 1), yl = __shfl_up(st[1], 1);
        const double xr = __shfl_down(st[0], 1), yr = __shfl_down(st[1], 1);
        const int al = __shfl_up((int)alive, 1), ar = __shfl_down((int)alive, 1);
        // cell (n - 1, j): nodes n - 1 and n of rays j and j + 1
        const double xrp = __shfl_down(xp, 1), yrp = __shfl_down(yp, 1);
        bool pix = false, ring = false;
        if (n >= 1 && has_right && alive && ar) {
            const double cxmin = fmin(fmin(xp, xrp), fmin(st[0], xr));
            const double cxmax = fmax(fmax(xp, xrp), fmax(st[0], xr));
            const double cymin = fmin(fmin(yp, yrp), fmin(st[1], yr));
            const double cymax = fmax(fmax(yp, yrp), fmax(st[1], yr));
            pix = ceil((cxmin - P.x0) * P.inv_h) <= fmin(floor((cxmax - P.x0) * P.inv_h), (double)(P.nx - 1)) &&
                  ceil((cymin - P.y0) * P.inv_h) <= fmin(floor((cymax - P.y0) * P.inv_h), (double)(P.ny - 1)) &&
                  cxmax >= P.x0 && cymax >= P.y0;
            const double dxm = cxmin > 0.0 ? cxmin : (cxmax < 0.0 ? -cxmax : 0.0);
            const double dym = cymin > 0.0 ? cymin : (cymax < 0.0 ? -cymax : 0.0);
            const double dmin2 = dxm * dxm + dym * dym;
            const double dmax2 = fmax(cxmin * cxmin, cxmax * cxmax) + fmax(cymin * cymin, cymax * cymax);
            ring = dmin2 <= P.ring2_hi && dmax2 >= P.ring2_lo;
        }
        {
            const uint64_t mp = __ballot(pix), mr = __ballot(ring);
            const uint64_t id = cell_id(eb, n - 1, j);
            if (pix) lp[cp + __popcll(mp & below)] = id;
            if (ring) lr[cr + __popcll(mr & below)] = id;
            cp += __popcll(mp);
            cr += __popcll(mr);
        }
        if (own && alive) {
            const bool lo = j > 0 && al;
            const bool hi = j + 1 < P.nr && ar;
            // chord between the neighbours at equal travel time (FP64
            // differences); J and a = sqrt(c / (8 pi J)) in FP32, the
            // precision the amplitude tables are stored in
            double dx = 0.0, dy = 0.0;
            float chord = 0.0f;
            if (lo && hi) {
                dx = xr - xl;
                dy = yr - yl;
                chord = (float)P.inv_chord_full;
            } else if (hi) {
                dx = xr - st[0];
                dy = yr - st[1];
                chord = (float)P.inv_chord_half;
            } else if (lo) {
                dx = st[0] - xl;
                dy = st[1] - yl;
                chord = (float)P.inv_chord_half;
            }
            float Jv = sqrtf((float)(dx * dx + dy * dy)) * chord;
            if (Jv < (float)P.j_min) Jv = (float)P.j_min;
            const float amp = 1.0f / sqrtf((float)s0 * ((float)eight_pi * Jv));
            const size_t k = base + (size_t)n * P.nr;
            // nodes are written once and read by later passes: keep them
            // from displacing the field grid in L2
            __builtin_nontemporal_store(nd2{st[0], st[1]}, reinterpret_cast<nd2 *>(&XY[k]));
            __builtin_nontemporal_store(nf2{amp, (float)st[4]}, reinterpret_cast<nf2 *>(&AB[k]));
        }
        xp = st[0];
        yp = st[1];
        if (alive && (last || n == P.nmax)) {
            if (own) L[(size_t)eb * P.nr + j] = n;
            alive = false;
        }
        if (alive) {
            double k1[5], k2[5], k3[5], k4[5], t[5];
            {
                const double is = recip(s0), is2 = is * is;
                k1[0] = st[2] * is2;
                k1[1] = st[3] * is2;
                k1[2] = g0x * is;
                k1[3] = g0y * is;
                k1[4] = a0 * is;
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) t[q] = st[q] + hdt * k1[q];
            rhs(sa, P, t, fc, k2);
#pragma unroll
            for (int q = 0; q < 5; ++q) t[q] = st[q] + hdt * k2[q];
            rhs(sa, P, t, fc, k3);
#pragma unroll
            for (int q = 0; q < 5; ++q) t[q] = st[q] + dt * k3[q];
            rhs(sa, P, t, fc, k4);
#pragma unroll
            for (int q = 0; q < 5; ++q) st[q] = st[q] + sixth * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
            last = st[0] * st[0] + st[1] * st[1] > P.rdie2;
        }
    }
    if (lane == 0) {
        seg_px[seg] = cp;
        seg_rx[seg] = cr;
    }
}

// Arrival key of a candidate: the interpolated step index u = T / dtau in
// fixed point, floor(max(u, 0) 2^F), above the triangle index
// idx = 2 (n nr + j) + tri.  The minimum key is the first arrival, equal
// fixed-point values going to the first triangle in (n, j, tri) order: the
// smallest interpolated travel time, except that two times within one
// quantum dtau 2^-F of each other count as equal.
// ~0 marks an uncovered point (no key reaches it: the fixed-point part
// stays below 2^(64 - idx_bits) - 2^F).
__device__ __forceinline__ uint64_t arrival_key(const TP &P, double u, uint32_t idx) {
    const uint64_t q = u > 0.0 ? (uint64_t)floor(u * P.qscale) : 0ull;
    return (q << P.idx_bits) | (uint64_t)idx;
}

struct Tri {
    double ax, ay, e1x, e1y, e2x, e2y, det, inv_det;
    double xmin, xmax, ymin, ymax;
};

__device__ __forceinline__ bool make_tri(double ax, double ay, double bx, double by, double cx, double cy,
                                         Tri &t) {
    t.ax = ax; t.ay = ay;
    t.e1x = bx - ax; t.e1y = by - ay;
    t.e2x = cx - ax; t.e2y = cy - ay;
    t.det = t.e1x * t.e2y - t.e1y * t.e2x;
    if (t.det == 0.0) return false;
    t.inv_det = 1.0 / t.det;
    t.xmin = fmin(ax, fmin(bx, cx)); t.xmax = fmax(ax, fmax(bx, cx));
    t.ymin = fmin(ay, fmin(by, cy)); t.ymax = fmax(ay, fmax(by, cy));
    return true;
}

// barycentric test at (qx, qy); returns false when outside
__device__ __forceinline__ bool bary(const Tri &t, double px, double py, double tol, double &la, double &lb,
                                     double &lc) {
    double qx = px - t.ax, qy = py - t.ay;
    lb = (qx * t.e2y - qy * t.e2x) * t.inv_det;
    lc = (t.e1x * qy - t.e1y * qx) * t.inv_det;
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

// Pixel-centre index range of the bounding box of triangle (a, b, c),
// clamped to the grid; false when the box holds no pixel centre.
__device__ __forceinline__ bool px_range(const TP &P, const double2 &pa, const double2 &pb, const double2 &pc,
                                         int &ilo, int &ihi, int &jlo, int &jhi) {
    const double xmin = fmin(pa.x, fmin(pb.x, pc.x)), xmax = fmax(pa.x, fmax(pb.x, pc.x));
    const double ymin = fmin(pa.y, fmin(pb.y, pc.y)), ymax = fmax(pa.y, fmax(pb.y, pc.y));
    double flo = ceil((xmin - P.x0) * P.inv_h), fhi = floor((xmax - P.x0) * P.inv_h);
    double glo = ceil((ymin - P.y0) * P.inv_h), ghi = floor((ymax - P.y0) * P.inv_h);
    if (flo < 0.0) flo = 0.0;
    if (glo < 0.0) glo = 0.0;
    if (fhi > (double)(P.nx - 1)) fhi = (double)(P.nx - 1);
    if (ghi > (double)(P.ny - 1)) ghi = (double)(P.ny - 1);
    if (!(flo <= fhi && glo <= ghi)) return false;
    ilo = (int)flo;
    ihi = (int)fhi;
    jlo = (int)glo;
    jhi = (int)ghi;
    return true;
}

// Receivers that may lie in a triangle's bounding box: a conservative index
// range around the ring (the box lies in a disc of radius hd around its
// centre c, which subtends at most asin(hd/|c|) <= hd/(|c| - hd) from the
// origin), or the whole ring when that bound does not apply.
__device__ __forceinline__ bool rx_range(const TP &P, const Tri &t, int &rlo, int &rhi) {
    double dxm = t.xmin > 0.0 ? t.xmin : (t.xmax < 0.0 ? -t.xmax : 0.0);
    double dym = t.ymin > 0.0 ? t.ymin : (t.ymax < 0.0 ? -t.ymax : 0.0);
    double dmin = sqrt(dxm * dxm + dym * dym);
    double dmax = sqrt(fmax(t.xmin * t.xmin, t.xmax * t.xmax) + fmax(t.ymin * t.ymin, t.ymax * t.ymax));
    if (!(dmin >= 0.0) || !(dmax >= 0.0)) return false;  // NaN nodes: nothing to test
    if (dmin > P.R * (1.0 + 1e-9) || dmax < P.R * (1.0 - 1e-9)) return false;
    const double cx = 0.5 * (t.xmin + t.xmax), cy = 0.5 * (t.ymin + t.ymax);
    const double wx = t.xmax - t.xmin, wy = t.ymax - t.ymin;
    const double hd = 0.5 * sqrt(wx * wx + wy * wy);
    const double rc = sqrt(cx * cx + cy * cy);
    if (!(rc > 2.0 * hd)) {
        rlo = 0; rhi = P.m - 1;
        return true;
    }
    const double th = atan2(cy, cx), dth = hd / (rc - hd);
    const double w = 2.0 * M_PI / (double)P.m;
    const double flo = floor((th - dth) / w) - 1.0, fhi = ceil((th + dth) / w) + 1.0;
    if (!(fhi - flo + 1.0 < (double)P.m) || !(flo >= -2.0 * P.m) || !(fhi <= 2.0 * P.m)) {
        rlo = 0; rhi = P.m - 1;   // whole ring (also catches non-finite angles)
        return true;
    }
    rlo = (int)flo;
    rhi = (int)fhi;
    return true;
}

// Element positions, computed once per call.
__global__ void k_rx_pos(TP P, double2 *__restrict__ rxy) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P.m) return;
    const double th = 2.0 * M_PI * (double)r / (double)P.m;
    rxy[r] = make_double2(P.R * cos(th), P.R * sin(th));
}

// Pixel pass: every candidate (triangle, pixel) pair takes the atomic
// minimum of its arrival key.  A wave takes one chunk of kRasterChunk
// entries of one list segment (work item = segment x chunk; chunks past the
// segment's end return at once).  Per triangle, the candidate pixel range
// comes first and the determinant only when the range is not empty.
constexpr int kRasterChunk = 512;

__global__ void __launch_bounds__(256) k_raster_px(TP P, const double2 *__restrict__ XY, int64_t nseg, int64_t cap,
                                                   const uint64_t *__restrict__ list, const int *__restrict__ segn,
                                                   uint64_t *__restrict__ akey) {
    const int64_t N = (int64_t)P.nx * P.ny;
    const double tol = -P.bary_tol;
    const int lane = threadIdx.x & 63;
    const int64_t nch = (cap + kRasterChunk - 1) / kRasterChunk;
    const int64_t item = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t seg = item / nch;
    if (seg >= nseg) return;
    const int i0 = (int)(item - seg * nch) * kRasterChunk;
    const int i1 = min(segn[seg], i0 + kRasterChunk);
    for (int i = i0 + lane; i < i1; i += 64) {
        int eb, n, j;
        cell_decode(list[seg * cap + i], eb, n, j);
        const int64_t base = (int64_t)eb * (P.nmax + 1) * P.nr;
        uint64_t *ak = akey + eb * N;
        for (int tri = 0; tri < 2; ++tri) {
            int64_t ka, kb, kc;
            int na, nb, nc;
            tri_nodes(base, n, j, P.nr, tri, ka, kb, kc, na, nb, nc);
            const double2 pa = XY[ka], pb = XY[kb], pc = XY[kc];
            int ilo, ihi, jlo, jhi;
            if (!px_range(P, pa, pb, pc, ilo, ihi, jlo, jhi)) continue;
            Tri t;
            if (!make_tri(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y, t)) continue;
            const double ua = (double)na, ub = (double)nb, uc = (double)nc;
            const uint32_t idx = ((uint32_t)n * (uint32_t)P.nr + (uint32_t)j) << 1 | (uint32_t)tri;
            for (int jj = jlo; jj <= jhi; ++jj) {
                for (int ii = ilo; ii <= ihi; ++ii) {
                    double la, lb, lc;
                    if (!bary(t, P.x0 + (double)ii * P.h, P.y0 + (double)jj * P.h, tol, la, lb, lc)) continue;
                    const uint64_t key = arrival_key(P, la * ua + lb * ub + lc * uc, idx);
                    atomicMin((unsigned long long *)&ak[(int64_t)jj * P.nx + ii], (unsigned long long)key);
                }
            }
        }
    }
}

// The same pass over the ring list, for the ring elements.
__global__ void __launch_bounds__(256) k_raster_rx(TP P, const double2 *__restrict__ XY, int64_t nseg, int64_t cap,
                                                   const uint64_t *__restrict__ list, const int *__restrict__ segn,
                                                   const double2 *__restrict__ rxy, uint64_t *__restrict__ akey_rx) {
    const double tol = -P.bary_tol;
    const int lane = threadIdx.x & 63;
    const int64_t nch = (cap + kRasterChunk - 1) / kRasterChunk;
    const int64_t item = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t seg = item / nch;
    if (seg >= nseg) return;
    const int i0 = (int)(item - seg * nch) * kRasterChunk;
    const int i1 = min(segn[seg], i0 + kRasterChunk);
    for (int i = i0 + lane; i < i1; i += 64) {
        int eb, n, j;
        cell_decode(list[seg * cap + i], eb, n, j);
        const int64_t base = (int64_t)eb * (P.nmax + 1) * P.nr;
        uint64_t *akr = akey_rx + (int64_t)eb * P.m;
        for (int tri = 0; tri < 2; ++tri) {
            int64_t ka, kb, kc;
            int na, nb, nc;
            tri_nodes(base, n, j, P.nr, tri, ka, kb, kc, na, nb, nc);
            Tri t;
            const double2 pa = XY[ka], pb = XY[kb], pc = XY[kc];
            if (!make_tri(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y, t)) continue;
            int rlo, rhi;
            if (!rx_range(P, t, rlo, rhi)) continue;
            const double ua = (double)na, ub = (double)nb, uc = (double)nc;
            const uint32_t idx = ((uint32_t)n * (uint32_t)P.nr + (uint32_t)j) << 1 | (uint32_t)tri;
            for (int rr = rlo; rr <= rhi; ++rr) {
                const int r = ((rr % P.m) + P.m) % P.m;
                const double2 q = rxy[r];
                if (q.x < t.xmin || q.x > t.xmax || q.y < t.ymin || q.y > t.ymax) continue;
                double la, lb, lc;
                if (!bary(t, q.x, q.y, tol, la, lb, lc)) continue;
                const uint64_t key = arrival_key(P, la * ua + lb * ub + lc * uc, idx);
                atomicMin((unsigned long long *)&akr[r], (unsigned long long)key);
            }
        }
    }
}

// Write pass: every point recomputes its first arrival's interpolation
// (the triangle index is the low part of its key) and writes T in place of
// the key, a and B.  Points are pixels (RX = false) or ring elements
// (RX = true).  With GS = float or double the pass writes the Green's
// tables of the frequency set (Gr, Gi [nf][m][N], `gofs` = e0 N) instead
// of T, a and B, from the same values (a and B rounded to float as the
// tables store them).
template <bool RX, typename GS = void>
__global__ void k_raster_write(TP P, const double2 *__restrict__ XY, const float2 *__restrict__ AB,
                               const double2 *__restrict__ rxy, uint64_t *__restrict__ akey,
                               float *__restrict__ amp_out, float *__restrict__ att_out,
                               uint8_t *__restrict__ cover, GreenParams GP = GreenParams(),
                               GS *__restrict__ Gr = nullptr, GS *__restrict__ Gi = nullptr, int64_t gofs = 0) {
    constexpr bool GREEN = !std::is_void<GS>::value;
    const int64_t npts = RX ? (int64_t)P.m : (int64_t)P.nx * P.ny;
    {
        // one flat grid over (emitter, point block), XCD-contiguous.  Pixel
        // blocks are 16 x 16 tiles, each wave an 8 x 8 square: neighbouring
        // lanes then interpolate on neighbouring mesh nodes whatever the ray
        // direction, so their gathers share cache lines.
        const int tx = (P.nx + 15) >> 4, ty = (P.ny + 15) >> 4;
        const int64_t bpe = RX ? (npts + 255) / 256 : (int64_t)tx * ty;
        const int64_t wg = xcd_remap(blockIdx.x, gridDim.x);
        const int eb = (int)(wg / bpe);
        const int64_t b = wg - (int64_t)eb * bpe;
        int64_t p;
        int ii = 0, jj = 0;
        if (RX) {
            p = b * 256 + threadIdx.x;
            if (p >= npts) return;
        } else {
            const int t = threadIdx.x, w = t >> 6, l = t & 63;
            const int by = (int)(b / tx), bx = (int)(b - (int64_t)by * tx);
            ii = bx * 16 + 8 * (w & 1) + (l & 7);
            jj = by * 16 + 8 * (w >> 1) + (l >> 3);
            if (ii >= P.nx || jj >= P.ny) return;
            p = (int64_t)jj * P.nx + ii;
        }
        const int64_t idx = (int64_t)eb * npts + p;
        const uint64_t key = akey[idx];
        double *Tout = reinterpret_cast<double *>(akey);
        const int64_t gstride = (int64_t)P.m * npts;   // one frequency of G
        auto uncovered = [&]() {
            if constexpr (GREEN) {
                for (int k = 0; k < GP.nf; ++k) {
                    Gr[k * gstride + gofs + idx] = GS(0.0f);
                    Gi[k * gstride + gofs + idx] = GS(0.0f);
                }
            } else {
                Tout[idx] = __longlong_as_double(0x7ff8000000000000ll);
                amp_out[idx] = 0.0f;
                att_out[idx] = 0.0f;
            }
            if (cover) cover[p] = 0;   // every writer stores the same value
        };
        if (key == ~0ull) {
            uncovered();
            return;
        }
        const uint32_t w = (uint32_t)(key & ((1ull << P.idx_bits) - 1ull));
        const int tri = (int)(w & 1u);
        const uint32_t cell = w >> 1;
        const int n = (int)(cell / (uint32_t)P.nr);
        const int j = (int)(cell - (uint32_t)n * (uint32_t)P.nr);
        if (n >= P.nmax || j >= P.nr - 1) {  // cannot occur for a key written by the pixel pass
            uncovered();
            return;
        }
        const int64_t base = (int64_t)eb * (P.nmax + 1) * P.nr;
        int64_t ka, kb, kc;
        int na, nb, nc;
        tri_nodes(base, n, j, P.nr, tri, ka, kb, kc, na, nb, nc);
        Tri t;
        const double2 pa = XY[ka], pb = XY[kb], pc = XY[kc];
        make_tri(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y, t);
        double px, py;
        if (RX) {
            const double2 q = rxy[p];
            px = q.x;
            py = q.y;
        } else {
            px = P.x0 + (double)ii * P.h;
            py = P.y0 + (double)jj * P.h;
        }
        double la, lb, lc;
        bary(t, px, py, -P.bary_tol, la, lb, lc);
        const double ta = (double)na * P.dtau, tb = (double)nb * P.dtau, tc = (double)nc * P.dtau;
        const double tv = la * ta + lb * tb + lc * tc;
        const float2 qa = AB[ka], qb = AB[kb], qc = AB[kc];
        const float av = (float)(la * (double)qa.x + lb * (double)qb.x + lc * (double)qc.x);
        const float bv = (float)(la * (double)qa.y + lb * (double)qb.y + lc * (double)qc.y);
        if constexpr (GREEN) {
            for (int k = 0; k < GP.nf; ++k) {
                double re, im;
                if constexpr (std::is_same<GS, __hip_bfloat16>::value) {
                    // BF16 tables hold G / omega^-1/2 (scale rsq per
                    // frequency): BF16 keeps FP32's exponent range, so no
                    // normalisation by the largest amplitude is needed
                    green_value_mag32(GP, k, tv, av, bv, re, im);
                    Gr[k * gstride + gofs + idx] = __float2bfloat16((float)re);
                    Gi[k * gstride + gofs + idx] = __float2bfloat16((float)im);
                } else {
                    green_value(GP, k, tv, (double)av * GP.rsq[k], (double)bv, re, im);
                    Gr[k * gstride + gofs + idx] = (GS)re;
                    Gi[k * gstride + gofs + idx] = (GS)im;
                }
            }
        } else {
            Tout[idx] = tv;
            amp_out[idx] = av;
            att_out[idx] = bv;
        }
    }
}

// Cell lists: one segment per tracing wave (batch emitter x wave), each
// with room for every cell of the wave's 62 owned rays.
inline int trace_waves(const rb_trace_opts *t) { return (t->n_rays + kOwn - 1) / kOwn; }
inline int64_t cell_seg_cap(const rb_trace_opts *t) { return (int64_t)kOwn * trace_nmax(t); }
inline int64_t cell_segments(const rb_trace_opts *t, int batch) { return (int64_t)trace_waves(t) * batch; }
inline unsigned raster_blocks(const rb_trace_opts *t, int batch) {
    const int64_t nch = (cell_seg_cap(t) + kRasterChunk - 1) / kRasterChunk;
    return (unsigned)((cell_segments(t, batch) * nch + 3) / 4);
}

struct TraceWs {
    double2 *sa, *rxy;
    double2 *XY;   // node position (x, y)
    float2 *AB;    // node (amplitude factor, absorption)
    int *L;
    uint64_t *list_px, *list_rx;  // candidate cells (pixel / ring), one segment per tracing wave
    int *seg_px, *seg_rx;         // segment lengths
};

size_t per_emitter_bytes(const rb_geometry *g, const rb_trace_opts *t) {
    (void)g;
    const size_t nodes = (size_t)(trace_nmax(t) + 1) * t->n_rays;
    const size_t segs = (size_t)cell_segments(t, 1);
    return nodes * (sizeof(double2) + sizeof(float2)) + (size_t)t->n_rays * sizeof(int) +
           2 * segs * ((size_t)cell_seg_cap(t) * sizeof(uint64_t) + sizeof(int)) + 10 * 256;
}

TraceWs carve_trace(Carver &c, const rb_geometry *g, const rb_trace_opts *t, int batch) {
    TraceWs w;
    const size_t nodes = (size_t)(trace_nmax(t) + 1) * t->n_rays * batch;
    w.sa = c.take<double2>((size_t)(g->nx + 4) * (g->ny + 4));
    w.rxy = c.take<double2>((size_t)g->m);
    w.XY = c.take<double2>(nodes);
    w.AB = c.take<float2>(nodes);
    w.L = c.take<int>((size_t)t->n_rays * batch);
    const size_t segs = (size_t)cell_segments(t, batch);
    w.list_px = c.take<uint64_t>(segs * (size_t)cell_seg_cap(t));
    w.list_rx = c.take<uint64_t>(segs * (size_t)cell_seg_cap(t));
    w.seg_px = c.take<int>(segs);
    w.seg_rx = c.take<int>(segs);
    return w;
}

TP make_tp(const rb_geometry *g, const rb_trace_opts *t) {
    TP P;
    P.nx = g->nx; P.ny = g->ny; P.h = g->h; P.x0 = g->x0; P.y0 = g->y0;
    P.inv_h = 1.0 / g->h;
    P.m = g->m; P.R = g->ring_radius; P.s_bg = 1.0 / g->c_background;
    P.nr = t->n_rays; P.dtau = t->dtau; P.nmax = (int)trace_nmax(t);
    const double r_die = g->ring_radius + 2.0 * g->h;
    P.rdie2 = r_die * r_die;
    P.j_min = t->j_min > 0.0 ? t->j_min : 0.25 * g->h;
    P.bary_tol = 1e-12;
    const double dpsi = M_PI / (double)t->n_rays;
    P.inv_chord_full = 1.0 / (2.0 * std::sin(dpsi));
    P.inv_chord_half = 1.0 / (2.0 * std::sin(0.5 * dpsi));
    P.ring2_lo = (g->ring_radius * (1.0 - 2e-9)) * (g->ring_radius * (1.0 - 2e-9));
    P.ring2_hi = (g->ring_radius * (1.0 + 2e-9)) * (g->ring_radius * (1.0 + 2e-9));
    {
        // arrival keys: triangle index in the low bits, fixed-point step index above
        auto bit_length = [](uint64_t v) { int b = 0; while (v) { ++b; v >>= 1; } return b; };
        const uint64_t nidx = 2ull * (uint64_t)P.nmax * (uint64_t)P.nr;
        P.idx_bits = bit_length(nidx - 1);
        P.qscale = std::ldexp(1.0, 64 - P.idx_bits - bit_length((uint64_t)P.nmax));
    }
    P.e0 = 0;
    P.ne = 0;
    return P;
}

}  // namespace

size_t trace_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t, int batch) {
    if (check_trace(g, t) != RB_OK) return 0;
    if (batch <= 0 || batch > g->m) batch = g->m;
    Carver c(nullptr, 0);
    carve_trace(c, g, t, batch);
    return c.used + 256;
}

// Traces all emitters into `out`, in batches that fit the workspace.  If
// `cover` is given, cover[p] is set to 0 for every pixel that some emitter
// does not reach (T = NaN) and left alone otherwise.  If `gout` is given,
// the pixel tables are not written: the write pass produces the Green's
// tables of `gout` instead (out->T still serves as the key buffer).
rb_status trace_rays_impl(const rb_geometry *g, const rb_trace_opts *t, const double *slowness,
                          const double *alpha0, const rb_tables *out, void *ws, size_t ws_bytes,
                          hipStream_t st, uint8_t *cover, const GreenOut *gout) {
    const int64_t N = (int64_t)g->nx * g->ny;
    // how many emitters fit
    Carver probe(nullptr, 0);
    carve_trace(probe, g, t, 1);
    const size_t one = probe.used + 256;
    if (ws_bytes < one) {
        set_error("trace workspace too small: need >= %zu bytes, got %zu", one, ws_bytes);
        return RB_ENOMEM;
    }
    // largest batch whose carve fits (estimate from above, then step down)
    int batch = (int)std::min<size_t>((size_t)g->m, 2 + (ws_bytes - one) / (per_emitter_bytes(g, t) - 10 * 256));
    while (batch > 1) {
        Carver c2(nullptr, 0);
        carve_trace(c2, g, t, batch);
        if (c2.used + 256 <= ws_bytes) break;
        --batch;
    }
    char *base = reinterpret_cast<char *>(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    Carver c(base, ws_bytes - (size_t)(base - (char *)ws));
    TraceWs w = carve_trace(c, g, t, batch);
    TP P = make_tp(g, t);
    const int64_t npad = (int64_t)(g->nx + 4) * (g->ny + 4);
    k_pack<<<blocks_for(npad, 256), 256, 0, st>>>(g->nx, g->ny, 1.0 / g->c_background, slowness, alpha0, w.sa);
    RB_LAUNCHED();
    k_rx_pos<<<blocks_for(g->m, 256), 256, 0, st>>>(P, w.rxy);
    RB_LAUNCHED();
    for (int e0 = 0; e0 < g->m; e0 += batch) {
        P.e0 = e0;
        P.ne = std::min(batch, g->m - e0);
        // the T tables hold the arrival keys until the write pass
        uint64_t *akey = reinterpret_cast<uint64_t *>(out->T + (int64_t)e0 * N);
        uint64_t *akey_rx = reinterpret_cast<uint64_t *>(out->T_rx + (int64_t)e0 * g->m);
        RB_TRY(fill_u64(akey, ~0ull, (int64_t)P.ne * N, st));
        RB_TRY(fill_u64(akey_rx, ~0ull, (int64_t)P.ne * g->m, st));
        const int64_t cap = cell_seg_cap(t);
        const int64_t nseg = cell_segments(t, P.ne);
        dim3 gt((trace_waves(t) + 3) / 4, P.ne);
        k_trace<<<gt, 256, 0, st>>>(P, w.sa, w.XY, w.AB, w.L, cap, w.list_px, w.list_rx, w.seg_px, w.seg_rx);
        RB_LAUNCHED();
        const unsigned nbl = raster_blocks(t, P.ne);
        k_raster_px<<<nbl, 256, 0, st>>>(P, w.XY, nseg, cap, w.list_px, w.seg_px, akey);
        RB_LAUNCHED();
        k_raster_rx<<<nbl, 256, 0, st>>>(P, w.XY, nseg, cap, w.list_rx, w.seg_rx, w.rxy, akey_rx);
        RB_LAUNCHED();
        const unsigned gw = (unsigned)(((g->nx + 15) / 16) * ((g->ny + 15) / 16)) * P.ne;
        if (gout && gout->dt == RB_F32)
            k_raster_write<false, float><<<gw, 256, 0, st>>>(P, w.XY, w.AB, w.rxy, akey, nullptr, nullptr, cover,
                                                             gout->P, (float *)gout->Gr, (float *)gout->Gi,
                                                             (int64_t)e0 * N);
        else if (gout && gout->dt == RB_BF16)
            k_raster_write<false, __hip_bfloat16><<<gw, 256, 0, st>>>(
                P, w.XY, w.AB, w.rxy, akey, nullptr, nullptr, cover, gout->P, (__hip_bfloat16 *)gout->Gr,
                (__hip_bfloat16 *)gout->Gi, (int64_t)e0 * N);
        else if (gout)
            k_raster_write<false, double><<<gw, 256, 0, st>>>(P, w.XY, w.AB, w.rxy, akey, nullptr, nullptr, cover,
                                                              gout->P, (double *)gout->Gr, (double *)gout->Gi,
                                                              (int64_t)e0 * N);
        else
            k_raster_write<false><<<gw, 256, 0, st>>>(P, w.XY, w.AB, w.rxy, akey, out->amp + (int64_t)e0 * N,
                                                      out->att + (int64_t)e0 * N, cover);
        RB_LAUNCHED();
        const unsigned gr = blocks_for(g->m, 256) * P.ne;
        k_raster_write<true><<<gr, 256, 0, st>>>(P, w.XY, w.AB, w.rxy, akey_rx, out->amp_rx + (int64_t)e0 * g->m,
                                                 out->att_rx + (int64_t)e0 * g->m, nullptr);
        RB_LAUNCHED();
    }
    return RB_OK;
}

// ------------------------------------------------------------- ToF model
// Bent-ray time-of-flight inversion for the starting model (Results
// section: a low-resolution image from three iterations of a ToF-based
// method that fits measured ToFs with ToFs modelled along rays).  The
// modelled ToF is the first-arrival time at a ring element; its linking
// path is read from the first-arrival triangle there: rays j and j + 1 of
// the cell, weighted 1 - w and w by the element's barycentrics, from the
// emitter to the step index u of the arrival.  Fermat's principle gives the
// linearisation dT = integral of ds along the path, with ds bilinear in the
// pixel values; along each polyline every point carries half of its two
// adjacent segment lengths (trapezoid rule).
namespace {

constexpr int kTofRB = kReduceBlocks;

__global__ void k_tof_slowness(const double *__restrict__ c, int64_t n, double *__restrict__ s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) s[i] = 1.0 / c[i];
}

// Per ordered pair (e, r): modelled ToF from the arrival key, the linking
// path (j, u, w; j = -1 if the pair is not used) and the residual
// dT = T_meas - T on the used pairs (selected, measured, covered), with
// used[] = 1.0 / 0.0.
__global__ void k_tof_link(TP P, int dmin, const double2 *__restrict__ XY, const double2 *__restrict__ rxy,
                           const uint64_t *__restrict__ akey_rx, const double *__restrict__ T_meas,
                           int *__restrict__ lj, double2 *__restrict__ luw, double *__restrict__ dT,
                           double *__restrict__ used) {
    const int64_t mm = (int64_t)P.m * P.m;
    const int64_t pr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pr >= mm) return;
    const int e = (int)(pr / P.m), r = (int)(pr - (int64_t)e * P.m);
    const int d0 = e > r ? e - r : r - e;
    const int dist = d0 < P.m - d0 ? d0 : P.m - d0;
    const uint64_t key = akey_rx[pr];
    const double tm = T_meas[pr];
    int j = -1;
    double u = 0.0, w = 0.0, res = 0.0;
    if (dist >= dmin && key != ~0ull && isfinite(tm)) {
        const uint32_t wk = (uint32_t)(key & ((1ull << P.idx_bits) - 1ull));
        const int tri = (int)(wk & 1u);
        const uint32_t cell = wk >> 1;
        const int n = (int)(cell / (uint32_t)P.nr);
        const int jc = (int)(cell - (uint32_t)n * (uint32_t)P.nr);
        if (n < P.nmax && jc < P.nr - 1) {
            const int64_t base = (int64_t)e * (P.nmax + 1) * P.nr;
            int64_t ka, kb, kc;
            int na, nb, nc;
            tri_nodes(base, n, jc, P.nr, tri, ka, kb, kc, na, nb, nc);
            Tri t;
            const double2 pa = XY[ka], pb = XY[kb], pc = XY[kc];
            make_tri(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y, t);
            const double2 q = rxy[r];
            double la, lb, lc;
            bary(t, q.x, q.y, -P.bary_tol, la, lb, lc);
            const double tv = la * ((double)na * P.dtau) + lb * ((double)nb * P.dtau) + lc * ((double)nc * P.dtau);
            u = la * (double)na + lb * (double)nb + lc * (double)nc;
            u = fmin(fmax(u, 0.0), (double)(n + 1));
            w = tri == 0 ? lb + lc : lb;
            j = jc;
            res = tm - tv;
        }
    }
    lj[pr] = j;
    luw[pr] = make_double2(u, w);
    dT[pr] = res;
    used[pr] = j >= 0 ? 1.0 : 0.0;
}

// Point i of ray q's path to parameter u (K = floor(u) nodes, then the
// fractional end point).
__device__ __forceinline__ double2 tof_point(const double2 *__restrict__ XY, int64_t base, int nr, int q, int i,
                                             int K, double fr) {
    if (i <= K) return XY[base + (int64_t)i * nr + q];
    const double2 a = XY[base + (int64_t)K * nr + q], b = XY[base + (int64_t)(K + 1) * nr + q];
    return make_double2(a.x + fr * (b.x - a.x), a.y + fr * (b.y - a.y));
}

// One wave per pair.  SCATTER: g += L^T dT and C += L^T 1 in fixed point
// (below); otherwise Lv[pair] = L v (fixed-order wave sum).  Every lane walks one
// contiguous run of point indices on both rays of the path at once; the
// points go into two register accumulators keyed by grid cell, so the
// points that share a cell (two to three consecutive ones at a step of
// about half a pixel, and mostly the neighbouring ray's as well) reach
// memory as one atomic per corner.
struct TofAcc {
    int ci, cj;
    int idx[4];
    double ag[4], ac[4];
};

// The back-projection sums in 64-bit fixed point: each contribution is
// rounded to a multiple of 1 / scale (scale a power of two set from a bound
// on a pixel's total, the residuals taken relative to max |dT|) and added
// with an integer atomic.  Integer sums are exact and independent of their
// order, so g and C are bitwise the same on every call.
__device__ __forceinline__ void tof_fix_add(long long *__restrict__ q, double x, double scale) {
    atomicAdd(reinterpret_cast<unsigned long long *>(q), (unsigned long long)llrint(x * scale));
}

__device__ __forceinline__ void tof_acc_flush(TofAcc &a, long long *__restrict__ gq, long long *__restrict__ Cq,
                                              double scale) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (a.idx[c] < 0) continue;
        tof_fix_add(&gq[a.idx[c]], a.ag[c], scale);
        tof_fix_add(&Cq[a.idx[c]], a.ac[c], scale);
    }
}

__device__ __forceinline__ void tof_acc_open(const TP &P, TofAcc &a, int ci, int cj) {
    a.ci = ci;
    a.cj = cj;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int ii = ci + (c & 1), jj = cj + (c >> 1);
        a.idx[c] = (ii >= 0 && ii < P.nx && jj >= 0 && jj < P.ny) ? jj * P.nx + ii : -1;
        a.ag[c] = 0.0;
        a.ac[c] = 0.0;
    }
}

template <bool SCATTER>
__global__ void __launch_bounds__(256) k_tof_path(TP P, const double2 *__restrict__ XY, const int *__restrict__ lj,
                                                  const double2 *__restrict__ luw, const double *__restrict__ dT,
                                                  const double *__restrict__ dTmax, double scale,
                                                  long long *__restrict__ gq, long long *__restrict__ Cq,
                                                  const double *__restrict__ v, double *__restrict__ Lv) {
    const int lane = threadIdx.x & 63;
    const int64_t pr = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t mm = (int64_t)P.m * P.m;
    if (pr >= mm) return;   // wave-uniform
    const int j = lj[pr];
    if (j < 0) {
        if (!SCATTER && lane == 0) Lv[pr] = 0.0;
        return;
    }
    const int e = (int)(pr / P.m);
    const double2 uw = luw[pr];
    const double u = uw.x;
    const int K = (int)floor(u);
    const double fr = u - (double)K;
    const int npts = K + 1 + (fr > 0.0 ? 1 : 0);
    const int64_t base = (int64_t)e * (P.nmax + 1) * P.nr;
    // the residual relative to max |dT| (|res| <= 1)
    const double res = SCATTER ? (dTmax[0] > 0.0 ? dT[pr] / dTmax[0] : 0.0) : 0.0;
    const int per = (npts + 63) >> 6;
    const int i0 = lane * per, i1 = min(npts, i0 + per);
    const double wq[2] = {1.0 - uw.y, uw.y};
    double acc = 0.0;
    // two accumulators held in registers (no dynamic indexing)
    TofAcc A0, A1;
    A0.ci = A1.ci = INT_MIN;
    A0.cj = A1.cj = INT_MIN;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        A0.idx[c] = A1.idx[c] = -1;
        A0.ag[c] = A0.ac[c] = A1.ag[c] = A1.ac[c] = 0.0;
    }
    bool victim1 = false;   // A1 (else A0) is replaced next
    if (i0 < i1) {
        double2 pc[2];
        double lprev[2] = {0.0, 0.0};
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            pc[sd] = tof_point(XY, base, P.nr, j + sd, i0, K, fr);
            if (i0 > 0) {
                const double2 pp = tof_point(XY, base, P.nr, j + sd, i0 - 1, K, fr);
                lprev[sd] = sqrt((pc[sd].x - pp.x) * (pc[sd].x - pp.x) + (pc[sd].y - pp.y) * (pc[sd].y - pp.y));
            }
        }
        for (int i = i0; i < i1; ++i) {
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                double lnext = 0.0;
                double2 pn = pc[sd];
                if (i + 1 < npts) {
                    pn = tof_point(XY, base, P.nr, j + sd, i + 1, K, fr);
                    lnext = sqrt((pn.x - pc[sd].x) * (pn.x - pc[sd].x) + (pn.y - pc[sd].y) * (pn.y - pc[sd].y));
                }
                const double f = wq[sd] * (0.5 * lprev[sd] + 0.5 * lnext);
                // bilinear weights of the four pixel centres around the point
                const double uu = (pc[sd].x - P.x0) * P.inv_h, vv = (pc[sd].y - P.y0) * P.inv_h;
                const double fi = floor(uu), fj = floor(vv);
                const double fu = uu - fi, fv = vv - fj;
                const int ci = (int)fmax(fmin(fi, 1e9), -1e9), cj = (int)fmax(fmin(fj, 1e9), -1e9);
                const double wt[4] = {(1.0 - fu) * (1.0 - fv), fu * (1.0 - fv), (1.0 - fu) * fv, fu * fv};
                if (SCATTER) {
                    bool use1;
                    if (A0.ci == ci && A0.cj == cj) {
                        use1 = false;
                    } else if (A1.ci == ci && A1.cj == cj) {
                        use1 = true;
                    } else {
                        use1 = victim1;
                        if (use1) {
                            tof_acc_flush(A1, gq, Cq, scale);
                            tof_acc_open(P, A1, ci, cj);
                        } else {
                            tof_acc_flush(A0, gq, Cq, scale);
                            tof_acc_open(P, A0, ci, cj);
                        }
                    }
                    victim1 = !use1;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const double x = f * wt[c];
                        A0.ag[c] += use1 ? 0.0 : x * res;
                        A0.ac[c] += use1 ? 0.0 : x;
                        A1.ag[c] += use1 ? x * res : 0.0;
                        A1.ac[c] += use1 ? x : 0.0;
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int ii = ci + (c & 1), jj = cj + (c >> 1);
                        if (ii >= 0 && ii < P.nx && jj >= 0 && jj < P.ny) acc += f * wt[c] * v[jj * P.nx + ii];
                    }
                }
                lprev[sd] = lnext;
                pc[sd] = pn;
            }
        }
    }
    if (SCATTER) {
        tof_acc_flush(A0, gq, Cq, scale);
        tof_acc_flush(A1, gq, Cq, scale);
    } else {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) Lv[pr] = acc;
    }
}

// g = gq / scale * max |dT|, C = Cq / scale (scale a power of two: exact
// divisions).
__global__ void k_tof_unfix(int64_t N, const long long *__restrict__ gq, const long long *__restrict__ Cq,
                            const double *__restrict__ dTmax, double scale, double *__restrict__ g,
                            double *__restrict__ C) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    g[x] = (double)gq[x] / scale * dTmax[0];
    C[x] = (double)Cq[x] / scale;
}

// Support: inside |x| < R - margin and crossed by some used path (C > 0).
__global__ void k_tof_support(TP P, double rs, const double *__restrict__ C, uint8_t *__restrict__ S) {
    const int64_t N = (int64_t)P.nx * P.ny;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t jj = p / P.nx, ii = p - jj * P.nx;
    const double px = P.x0 + (double)ii * P.h, py = P.y0 + (double)jj * P.h;
    S[p] = (px * px + py * py < rs * rs && C[p] > 0.0) ? 1 : 0;
}

__global__ void k_tof_direction(int64_t n, const double *__restrict__ g, const double *__restrict__ C,
                                const uint8_t *__restrict__ S, const double *__restrict__ cmax, double eps,
                                double *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double cm = cmax[0] > -INFINITY ? cmax[0] : 0.0;
    v[i] = S[i] ? g[i] / (C[i] + eps * cm) : 0.0;
}

// Fixed-order block sums of a.b, b.b and a.a over [0, n): part[3 b + 0..2].
__global__ void k_tof_sums(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                           double *__restrict__ part) {
    __shared__ double s0[256], s1[256], s2[256];
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double ai = a[i], bi = b[i];
        x0 += ai * bi;
        x1 += bi * bi;
        x2 += ai * ai;
    }
    s0[threadIdx.x] = x0;
    s1[threadIdx.x] = x1;
    s2[threadIdx.x] = x2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s0[threadIdx.x] += s0[threadIdx.x + st];
            s1[threadIdx.x] += s1[threadIdx.x + st];
            s2[threadIdx.x] += s2[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s0[0];
        part[3 * blockIdx.x + 1] = s1[0];
        part[3 * blockIdx.x + 2] = s2[0];
    }
}

// res[slot + 0..2] = the three sums.
__global__ void k_tof_sums_final(const double *__restrict__ part, int np, double *__restrict__ res, int slot) {
    __shared__ double s0[256], s1[256], s2[256];
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) {
        x0 += part[3 * i];
        x1 += part[3 * i + 1];
        x2 += part[3 * i + 2];
    }
    s0[threadIdx.x] = x0;
    s1[threadIdx.x] = x1;
    s2[threadIdx.x] = x2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s0[threadIdx.x] += s0[threadIdx.x + st];
            s1[threadIdx.x] += s1[threadIdx.x + st];
            s2[threadIdx.x] += s2[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        res[slot] = s0[0];
        res[slot + 1] = s1[0];
        res[slot + 2] = s2[0];
    }
}

// res: [1] sum dT^2, [2] number of used pairs (the (used, dT) sums);
// [3] <Lv, dT>, [5] <Lv, Lv> (the (Lv, dT) sums).  The update check counts
// the pixels with s + beta v <= 0, beta = res[3] / res[5].
__global__ void k_tof_update_check(int64_t n, const double *__restrict__ s, const double *__restrict__ v,
                                   double *__restrict__ res, double *__restrict__ part) {
    __shared__ double sb[256];
    const double beta = res[5] > 0.0 ? res[3] / res[5] : 0.0;
    double bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double ds = beta * v[i];
        if (ds != 0.0 && !(s[i] + ds > 0.0)) bad += 1.0;
    }
    sb[threadIdx.x] = bad;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sb[threadIdx.x] += sb[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sb[0];
}

// res[6] = beta, res[7] = number of failed pixels
__global__ void k_tof_update_final(const double *__restrict__ part, int np, double *__restrict__ res) {
    __shared__ double sb[256];
    double bad = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) bad += part[i];
    sb[threadIdx.x] = bad;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sb[threadIdx.x] += sb[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        res[6] = res[5] > 0.0 ? res[3] / res[5] : 0.0;
        res[7] = sb[0];
    }
}

// c = 1 / (s + beta v) where beta v != 0, if no pixel failed the check.
__global__ void k_tof_update_write(int64_t n, const double *__restrict__ s, const double *__restrict__ v,
                                   const double *__restrict__ res, double *__restrict__ c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || res[7] != 0.0) return;
    const double ds = res[6] * v[i];
    if (ds != 0.0) c[i] = 1.0 / (s[i] + ds);
}

struct TofWs {
    double *c, *s, *g, *C, *v, *dT, *used, *Lv, *part, *res, *cmax, *dTmax;
    long long *gq, *Cq;   // g, C in fixed point
    double2 *luw;
    int *lj;
    uint8_t *S;
    uint64_t *akey_rx;
    TraceWs tw;
};

TofWs carve_tof(Carver &c, const rb_geometry *g, const rb_trace_opts *t) {
    const size_t N = (size_t)g->nx * g->ny, mm = (size_t)g->m * g->m;
    TofWs w;
    w.c = c.take<double>(N);
    w.s = c.take<double>(N);
    w.g = c.take<double>(N);
    w.C = c.take<double>(N);
    w.v = c.take<double>(N);
    w.S = c.take<uint8_t>(N);
    w.dT = c.take<double>(mm);
    w.used = c.take<double>(mm);
    w.Lv = c.take<double>(mm);
    w.luw = c.take<double2>(mm);
    w.lj = c.take<int>(mm);
    w.akey_rx = c.take<uint64_t>(mm);
    w.part = c.take<double>(3 * kTofRB);
    w.res = c.take<double>(8);
    w.cmax = c.take<double>(1);
    w.dTmax = c.take<double>(1);
    w.gq = c.take<long long>(N);
    w.Cq = c.take<long long>(N);
    w.tw = carve_trace(c, g, t, g->m);   // every emitter's fan stays resident
    return w;
}

}  // namespace

size_t tof_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t) {
    Carver c(nullptr, 0);
    carve_tof(c, g, t);
    return c.used + 256;
}

// n_iter linearised ToF iterations from c_in; hist [host][2 n_iter] (nullable)
// receives (rms dT before the update, beta) per iteration.
rb_status tof_invert_impl(const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o,
                          const double *c_in, const double *T_meas, int n_iter, double *c_out, double *hist,
                          void *ws, size_t ws_bytes, hipStream_t st) {
    if (tof_workspace_bytes(g, t) > ws_bytes) {
        set_error("ToF workspace too small: need %zu bytes, got %zu", tof_workspace_bytes(g, t), ws_bytes);
        return RB_ENOMEM;
    }
    char *base = reinterpret_cast<char *>(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    Carver cv(base, ws_bytes - (size_t)(base - (char *)ws));
    TofWs w = carve_tof(cv, g, t);
    TP P = make_tp(g, t);
    P.e0 = 0;
    P.ne = g->m;
    const int64_t N = (int64_t)g->nx * g->ny;
    const int m = g->m;
    const int64_t mm = (int64_t)m * m;
    const int dmin = (int)std::ceil((1.0 - o->recv_fraction) * 0.5 * m - 1e-9);
    const double rs = g->ring_radius - g->support_margin;
    // fixed-point scale of the back-projection: a used pair adds at most
    // about 4h of weighted path length to a pixel (two rays, weights summing
    // to 1, the path's length inside the pixel's bilinear support plus half
    // a step at either end), and |dT / max|dT|| <= 1, so |g|, |C| <= 4 h m^2
    // in those units; twice that stays below 2^60 / scale
    const double fix_scale = std::ldexp(1.0, 60 - (int)std::ceil(std::log2(8.0 * g->h * (double)mm)));
    RB_HIP(hipMemcpyAsync(w.c, c_in, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    k_rx_pos<<<blocks_for(m, 256), 256, 0, st>>>(P, w.tw.rxy);
    RB_LAUNCHED();
    const int64_t npad = (int64_t)(g->nx + 4) * (g->ny + 4);
    const int64_t cap = cell_seg_cap(t);
    const int64_t nseg = cell_segments(t, m);
    for (int it = 0; it < n_iter; ++it) {
        // rays and first arrivals at the ring elements in the current model
        k_tof_slowness<<<blocks_for(N, 256), 256, 0, st>>>(w.c, N, w.s);
        RB_LAUNCHED();
        k_pack<<<blocks_for(npad, 256), 256, 0, st>>>(g->nx, g->ny, P.s_bg, w.s, nullptr, w.tw.sa);
        RB_LAUNCHED();
        RB_TRY(fill_u64(w.akey_rx, ~0ull, mm, st));
        k_trace<<<dim3((trace_waves(t) + 3) / 4, m), 256, 0, st>>>(P, w.tw.sa, w.tw.XY, w.tw.AB, w.tw.L, cap,
                                                                 w.tw.list_px, w.tw.list_rx, w.tw.seg_px,
                                                                 w.tw.seg_rx);
        RB_LAUNCHED();
        k_raster_rx<<<raster_blocks(t, m), 256, 0, st>>>(P, w.tw.XY, nseg, cap, w.tw.list_rx, w.tw.seg_rx,
                                                          w.tw.rxy, w.akey_rx);
        RB_LAUNCHED();
        // linking paths and residuals
        k_tof_link<<<blocks_for(mm, 256), 256, 0, st>>>(P, dmin, w.tw.XY, w.tw.rxy, w.akey_rx, T_meas, w.lj,
                                                         w.luw, w.dT, w.used);
        RB_LAUNCHED();
        k_tof_sums<<<kTofRB, 256, 0, st>>>(mm, w.used, w.dT, w.part);
        RB_LAUNCHED();
        k_tof_sums_final<<<1, 256, 0, st>>>(w.part, kTofRB, w.res, 0);   // res[1] sum dT^2, [2] used pairs
        RB_LAUNCHED();
        // back-projection of the residuals and the ray density, in fixed point
        RB_TRY(reduce_absmax_f64(w.dT, mm, w.part, w.dTmax, st));
        RB_TRY(fill_u64(reinterpret_cast<uint64_t *>(w.gq), 0ull, N, st));
        RB_TRY(fill_u64(reinterpret_cast<uint64_t *>(w.Cq), 0ull, N, st));
        const unsigned gp = (unsigned)((mm + 3) / 4);
        k_tof_path<true><<<gp, 256, 0, st>>>(P, w.tw.XY, w.lj, w.luw, w.dT, w.dTmax, fix_scale, w.gq, w.Cq,
                                              nullptr, nullptr);
        RB_LAUNCHED();
        k_tof_unfix<<<blocks_for(N, 256), 256, 0, st>>>(N, w.gq, w.Cq, w.dTmax, fix_scale, w.g, w.C);
        RB_LAUNCHED();
        k_tof_support<<<blocks_for(N, 256), 256, 0, st>>>(P, rs, w.C, w.S);
        RB_LAUNCHED();
        RB_TRY(reduce_max_f64(w.C, w.S, N, w.part, w.cmax, st));
        k_tof_direction<<<blocks_for(N, 256), 256, 0, st>>>(N, w.g, w.C, w.S, w.cmax, o->eps, w.v);
        RB_LAUNCHED();
        // exact step along v
        k_tof_path<false><<<gp, 256, 0, st>>>(P, w.tw.XY, w.lj, w.luw, nullptr, nullptr, 0.0, nullptr, nullptr,
                                               w.v, w.Lv);
        RB_LAUNCHED();
        k_tof_sums<<<kTofRB, 256, 0, st>>>(mm, w.Lv, w.dT, w.part);
        RB_LAUNCHED();
        k_tof_sums_final<<<1, 256, 0, st>>>(w.part, kTofRB, w.res, 3);   // res[3] <Lv,dT>, [4] dT^2, [5] <Lv,Lv>
        RB_LAUNCHED();
        k_tof_update_check<<<kTofRB, 256, 0, st>>>(N, w.s, w.v, w.res, w.part);
        RB_LAUNCHED();
        k_tof_update_final<<<1, 256, 0, st>>>(w.part, kTofRB, w.res);
        RB_LAUNCHED();
        k_tof_update_write<<<blocks_for(N, 256), 256, 0, st>>>(N, w.s, w.v, w.res, w.c);
        RB_LAUNCHED();
        double res[8];
        RB_HIP(hipMemcpyAsync(res, w.res, sizeof(res), hipMemcpyDeviceToHost, st));
        RB_HIP(hipStreamSynchronize(st));
        if (hist) {
            hist[2 * it] = res[2] > 0.0 ? std::sqrt(res[1] / res[2]) : 0.0;
            hist[2 * it + 1] = res[6];
        }
        if (res[7] != 0.0) {
            set_error("slowness update not positive at %.0f pixels (iteration %d); c_out not written", res[7], it);
            return RB_ENUMERIC;
        }
    }
    RB_HIP(hipMemcpyAsync(c_out, w.c, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    RB_HIP(hipStreamSynchronize(st));
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
    return rb::trace_rays_impl(g, t, slowness, alpha0, out, ws, ws_bytes, rb::as_stream(stream), nullptr,
                               nullptr);
}

size_t rb_tof_workspace_bytes(const rb_geometry *g, const rb_trace_opts *t) {
    if (rb::check_trace(g, t) != RB_OK) return 0;
    return rb::tof_workspace_bytes(g, t);
}

rb_status rb_tof_invert(const rb_geometry *g, const rb_trace_opts *t, const rb_invert_opts *o,
                        const double *c_in, const double *T_meas, int32_t n_iter, double *c_out, double *hist,
                        void *ws, size_t ws_bytes, void *stream) {
    rb::clear_error();
    RB_TRY(rb::check_trace(g, t));
    RB_CHECK_ARG(o != nullptr, "invert options are NULL");
    RB_CHECK_ARG(o->recv_fraction > 0.0 && o->recv_fraction <= 1.0, "recv_fraction must be in (0, 1]");
    RB_CHECK_ARG(std::isfinite(o->eps) && o->eps >= 0.0, "eps must be >= 0");
    RB_CHECK_ARG(n_iter >= 1 && n_iter <= 64, "n_iter must be in [1, 64]");
    RB_CHECK_ARG(c_in && T_meas && c_out, "c_in/T_meas/c_out are NULL");
    RB_CHECK_ARG(ws != nullptr, "workspace is NULL");
    return rb::tof_invert_impl(g, t, o, c_in, T_meas, n_iter, c_out, hist, ws, ws_bytes, rb::as_stream(stream));
}

}  // extern "C"
