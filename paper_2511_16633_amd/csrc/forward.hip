// Born forward operator (paper, Inverse Problem section, Eqs. 8-9;
// linearisation of Eq. 1 in q = 1/c^2 with Green's functions from Eqs. 4-5).
//
//   d_er = omega^2 h^2 sum_x G_e(x) G_r(x) delta(x)
//
// A split-K complex GEMM over pixels on the matrix cores.  The output is
// symmetric in (e, r), so only upper-triangular tiles are computed; the
// split partials are reduced in a fixed order.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "born.h"
#include "common.h"
#include "mma.h"

namespace rb {
namespace {

// ------------------------------------------------------------------ forward
// Output tile 64x64 (e, r) with tile_e <= tile_r; wave w owns rows 16w..+15
// and four 16-column blocks; K = pixels [ks, ks + kchunk).
__device__ __forceinline__ void tri_tile(int t, int ntl, int &te, int &tr) {
    // enumerate (te, tr) with te <= tr row by row
    int a = 0;
    while (t >= ntl - a) {
        t -= ntl - a;
        ++a;
    }
    te = a;
    tr = a + t;
}

// Largest circular index distance min(|e - r|, m - |e - r|) over the pairs
// e in [e0, e0 + ne), r in [r0, r0 + nr): the distance is piecewise linear
// in r - e with its peaks at +-m/2, so the maximum is at an end of the
// difference range or at a peak inside it.
__device__ __forceinline__ int max_circ_dist(int m, int e0, int ne, int r0, int nr) {
    const int lo = r0 - (e0 + ne - 1), hi = (r0 + nr - 1) - e0;
    auto cd = [m](int d) {
        d = d < 0 ? -d : d;
        d %= m;
        return d < m - d ? d : m - d;
    };
    int best = cd(lo) > cd(hi) ? cd(lo) : cd(hi);
    const int h = m / 2;
    if ((lo <= h && h <= hi) || (lo <= -h && -h <= hi)) best = h;
    return best;
}

// A 32 x 32 (e, r) block of a tile whose value is never used: below the
// diagonal of a diagonal tile (the reduction reads e <= r), or, with
// dmin >= 32, every pair of the block closer than dmin (weighted by zero).
__device__ __forceinline__ bool fwd_block_idle(const FwdParams &P, int te, int tr, int we, int wr) {
    if (te == tr && we > wr) return true;
    return P.dmin >= 32 &&
           max_circ_dist(P.m, te * 64 + 32 * we, 32, tr * 64 + 32 * wr, 32) < P.dmin;
}

template <typename T>
__global__ void __launch_bounds__(256) k_forward(FwdParams P, const T *__restrict__ Gr, const T *__restrict__ Gi,
                                                 const double *__restrict__ delta, T *__restrict__ part) {
    using acc_t = typename MM<T>::acc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kk = lane >> 4;
    int te, tr;
    tri_tile(blockIdx.x, P.ntl, te, tr);
    const int split = blockIdx.y, k = blockIdx.z;
    const int64_t N = P.N;
    const T *gr = Gr + (int64_t)k * P.m * N;
    const T *gi = Gi + (int64_t)k * P.m * N;
    const int e = te * 64 + 16 * wave + row;
    const int64_t ks = (int64_t)split * P.kchunk;
    const int64_t ke = std::min<int64_t>(N, ks + P.kchunk);
    acc_t re[4], im[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) re[c] = im[c] = acc_t{0, 0, 0, 0};
    for (int64_t xc = ks; xc < ke; xc += 16) {
        T a_r[4], a_i[4], dl[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t x = xc + 4 * kk + s;
            const bool okx = x < ke;
            dl[s] = okx ? (T)delta[x] : T(0);
            a_r[s] = ld(gr + (int64_t)e * N + x, okx && e < P.m);
            a_i[s] = ld(gi + (int64_t)e * N + x, okx && e < P.m);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int r = tr * 64 + 16 * c + row;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int64_t x = xc + 4 * kk + s;
                const bool ok = (x < ke) && (r < P.m);
                const T b_r = ld(gr + (int64_t)r * N + x, ok) * dl[s];
                const T b_i = ld(gi + (int64_t)r * N + x, ok) * dl[s];
                re[c] = MM<T>::mma(a_r[s], b_r, re[c]);
                re[c] = MM<T>::mma(-a_i[s], b_i, re[c]);
                im[c] = MM<T>::mma(a_r[s], b_i, im[c]);
                im[c] = MM<T>::mma(a_i[s], b_r, im[c]);
            }
        }
    }
    // partial tile -> part[split][k][e][r][2]
    T *pp = part + ((int64_t)split * P.nf + k) * P.mp * P.mp * 2;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int r = tr * 64 + 16 * c + row;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ee = te * 64 + 16 * wave + MM<T>::out_row(kk, i);
            const int64_t o = ((int64_t)ee * P.mp + r) * 2;
            pp[o] = re[c][i];
            pp[o + 1] = im[c][i];
        }
    }
}

// d[k][e][r] = c_k * sum_split part (fixed order) over the upper triangle
// e <= r, written to (e, r) and (r, e).  A thread per upper-triangle entry of
// a row-major [mp][mp] index (entries below the diagonal exit), so the
// partial reads are coalesced; eight splits are loaded together.
template <typename T>
__global__ void k_forward_reduce(FwdParams P, const T *__restrict__ part, const float *__restrict__ gscale,
                                 const double *__restrict__ dmax, double *__restrict__ d) {
    const int64_t mm = (int64_t)P.m * P.m;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= mm * P.nf) return;
    const int k = (int)(idx / mm);
    const int64_t rem = idx - (int64_t)k * mm;
    const int e = (int)(rem / P.m), r = (int)(rem - (int64_t)e * P.m);
    if (e > r) return;
    if (P.dmin >= 32 && min(r - e, P.m - (r - e)) < P.dmin) {
        // weighted by zero by the caller; its tile may not have been computed
        const int64_t o1 = ((int64_t)k * P.m + e) * P.m + r, o2 = ((int64_t)k * P.m + r) * P.m + e;
        d[2 * o1] = d[2 * o1 + 1] = d[2 * o2] = d[2 * o2 + 1] = 0.0;
        return;
    }
    const int64_t stride = (int64_t)P.nf * P.mp * P.mp * 2;   // one split
    const T *pp = part + (int64_t)k * P.mp * P.mp * 2 + ((int64_t)e * P.mp + r) * 2;
    double sr = 0.0, si = 0.0;
    constexpr int kU = 8;
    for (int s0 = 0; s0 < P.nsplit; s0 += kU) {
        T vr[kU], vi[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const bool ok = s0 + u < P.nsplit;
            vr[u] = ok ? pp[(s0 + u) * stride] : T(0);
            vi[u] = ok ? pp[(s0 + u) * stride + 1] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (s0 + u < P.nsplit) {
                sr += (double)vr[u];
                si += (double)vi[u];
            }
        }
    }
    double c = P.cg[k];
    if (gscale) {
        const double g = (double)gscale[k];
        c *= g * g;
    }
    if (dmax) c *= dmax[0];
    const double vr = sr * c, vi = si * c;
    const int64_t o1 = ((int64_t)k * P.m + e) * P.m + r, o2 = ((int64_t)k * P.m + r) * P.m + e;
    d[2 * o1] = vr;
    d[2 * o1 + 1] = vi;
    d[2 * o2] = vr;
    d[2 * o2 + 1] = vi;
}

// Workgroup -> (tile, split, frequency) for the flat grid of the 16-bit
// kernel.  The tiles of one pixel split read the same pixel range of G, so
// consecutive logical ids (tile fastest) are kept on one XCD and its L2.
__device__ __forceinline__ void fwd_block(const FwdParams &P, int &te, int &tr, int &split, int &k) {
    const int64_t nblk = (int64_t)P.ntri * P.nsplit * P.nf;
    const int64_t L = xcd_remap(blockIdx.x, nblk);
    const int t = (int)(L % P.ntri);
    const int64_t rest = L / P.ntri;
    split = (int)(rest % P.nsplit);
    k = (int)(rest / P.nsplit);
    tri_tile(t, P.ntl, te, tr);
}

// Forward, tables whose rows are not 16-byte aligned (N not a multiple of
// 4).  A 64 x 64 (e, r) output tile per workgroup (upper triangle only)
// over a split of the pixels; waves are 2 x 2, each 32 e x 32 r.  Pixels are
// consumed 32 at a time: G_e and G_r delta for the tile's rows are staged in
// LDS as [row][32 px] (stride 36), double buffered through registers; a
// lane reads its eight k values of a row as two b128 reads.
constexpr int kFwdKC = 32, kFwdLD = 36;

// One thread's staging registers: eight pixels of one row of G_e and of
// G_r, and delta at those pixels.  G_r delta is formed when the tile is
// stored, not when it is loaded, so the loads stay in flight during the
// MFMAs of the current tile.
struct FwdStage {
    f4 ar[2], ai[2], br[2], bi[2];
    double dl[8];
};

__device__ __forceinline__ void fwd_stage_load(const float *__restrict__ gr, const float *__restrict__ gi,
                                               const double *__restrict__ delta, int m, int64_t N, int e_row,
                                               int r_row, int64_t xc, int64_t ke, bool vec, FwdStage &v) {
    const int c8 = (threadIdx.x & 3) * 8;
    const int64_t xs = xc + c8;
    if (vec) {
#pragma unroll
        for (int q = 0; q < 8; ++q) v.dl[q] = delta[xs + q];
        if (e_row < m) {
            const float *pr = gr + (int64_t)e_row * N + xs;
            const float *pi = gi + (int64_t)e_row * N + xs;
            v.ar[0] = *reinterpret_cast<const f4 *>(pr);
            v.ar[1] = *reinterpret_cast<const f4 *>(pr + 4);
            v.ai[0] = *reinterpret_cast<const f4 *>(pi);
            v.ai[1] = *reinterpret_cast<const f4 *>(pi + 4);
        } else {
            v.ar[0] = v.ar[1] = v.ai[0] = v.ai[1] = f4{0, 0, 0, 0};
        }
        if (r_row < m) {
            const float *pr = gr + (int64_t)r_row * N + xs;
            const float *pi = gi + (int64_t)r_row * N + xs;
            v.br[0] = *reinterpret_cast<const f4 *>(pr);
            v.br[1] = *reinterpret_cast<const f4 *>(pr + 4);
            v.bi[0] = *reinterpret_cast<const f4 *>(pi);
            v.bi[1] = *reinterpret_cast<const f4 *>(pi + 4);
        } else {
            v.br[0] = v.br[1] = v.bi[0] = v.bi[1] = f4{0, 0, 0, 0};
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t x = xs + q;
            const bool okx = x < ke;
            v.dl[q] = okx ? delta[x] : 0.0;
            const bool oka = okx && e_row < m, okb = okx && r_row < m;
            v.ar[q >> 2][q & 3] = oka ? gr[(int64_t)e_row * N + x] : 0.0f;
            v.ai[q >> 2][q & 3] = oka ? gi[(int64_t)e_row * N + x] : 0.0f;
            v.br[q >> 2][q & 3] = okb ? gr[(int64_t)r_row * N + x] : 0.0f;
            v.bi[q >> 2][q & 3] = okb ? gi[(int64_t)r_row * N + x] : 0.0f;
        }
    }
}

__global__ void __launch_bounds__(256, 2) k_forward_f32_regs(FwdParams P, const float *__restrict__ Gr,
                                                             const float *__restrict__ Gi,
                                                             const double *__restrict__ delta,
                                                             float *__restrict__ part) {
    __shared__ float sA[2][2][64][kFwdLD];
    __shared__ float sBm[2][2][64][kFwdLD];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kk = lane >> 4;
    const int we = wave >> 1, wr = wave & 1;
    int te, tr;
    tri_tile(blockIdx.x, P.ntl, te, tr);
    const int split = blockIdx.y, k = blockIdx.z;
    const int64_t N = P.N;
    const float *gr = Gr + (int64_t)k * P.m * N;
    const float *gi = Gi + (int64_t)k * P.m * N;
    const int64_t ks = (int64_t)split * P.kchunk;
    const int64_t ke = std::min<int64_t>(N, ks + P.kchunk);
    const int nch = (int)((ke - ks + kFwdKC - 1) / kFwdKC);
    const int srow = tid >> 2, c8 = (tid & 3) * 8;
    const int e_row = te * 64 + srow, r_row = tr * 64 + srow;
    // Waves whose block is never used only stage (wave-uniform); a tile
    // with no used block returns at once (the reduction does not read it).
    if (P.dmin >= 32 && max_circ_dist(P.m, te * 64, 64, tr * 64, 64) < P.dmin) return;
    const bool idle = fwd_block_idle(P, te, tr, we, wr);
    // (a + ib)(c + id) with three real products: P1 = ac, P2 = bd,
    // P3 = (a + b)(c + d); re = P1 - P2, im = P3 - P1 - P2
    f4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) p1[b][c] = p2[b][c] = p3[b][c] = f4{0, 0, 0, 0};
    auto vec_ok = [&](int64_t xc) { return ((N & 3) == 0) && (xc + kFwdKC <= ke); };
    auto store = [&](int buf, const FwdStage &stg) {
        *reinterpret_cast<f4 *>(&sA[buf][0][srow][c8]) = stg.ar[0];
        *reinterpret_cast<f4 *>(&sA[buf][0][srow][c8 + 4]) = stg.ar[1];
        *reinterpret_cast<f4 *>(&sA[buf][1][srow][c8]) = stg.ai[0];
        *reinterpret_cast<f4 *>(&sA[buf][1][srow][c8 + 4]) = stg.ai[1];
        f4 br0, br1, bi0, bi1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            br0[q] = stg.br[0][q] * (float)stg.dl[q];
            br1[q] = stg.br[1][q] * (float)stg.dl[q + 4];
            bi0[q] = stg.bi[0][q] * (float)stg.dl[q];
            bi1[q] = stg.bi[1][q] * (float)stg.dl[q + 4];
        }
        *reinterpret_cast<f4 *>(&sBm[buf][0][srow][c8]) = br0;
        *reinterpret_cast<f4 *>(&sBm[buf][0][srow][c8 + 4]) = br1;
        *reinterpret_cast<f4 *>(&sBm[buf][1][srow][c8]) = bi0;
        *reinterpret_cast<f4 *>(&sBm[buf][1][srow][c8 + 4]) = bi1;
    };
    auto load = [&](int c, FwdStage &v) {
        const int64_t xc = ks + (int64_t)c * kFwdKC;
        fwd_stage_load(gr, gi, delta, P.m, N, e_row, r_row, xc, ke, vec_ok(xc), v);
    };
    // Tiles are loaded two steps ahead into two register sets used in turn
    // (as in the 16-bit kernel); FUT: tile c + 2 exists and is whole.
    auto step = [&](int c, FwdStage &next, FwdStage &fut, auto fut_tag) {
        const int buf = c & 1;
        if (decltype(fut_tag)::value)
            fwd_stage_load(gr, gi, delta, P.m, N, e_row, r_row, ks + (int64_t)(c + 2) * kFwdKC, ke, true, fut);
        else if (c + 2 < nch)
            load(c + 2, fut);
        if (!idle) {
        f4 a_r[2][2], a_i[2][2], b_r[2][2], b_i[2][2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int ra = 32 * we + 16 * b + row;
            a_r[b][0] = *reinterpret_cast<const f4 *>(&sA[buf][0][ra][8 * kk]);
            a_r[b][1] = *reinterpret_cast<const f4 *>(&sA[buf][0][ra][8 * kk + 4]);
            a_i[b][0] = *reinterpret_cast<const f4 *>(&sA[buf][1][ra][8 * kk]);
            a_i[b][1] = *reinterpret_cast<const f4 *>(&sA[buf][1][ra][8 * kk + 4]);
            const int rb = 32 * wr + 16 * b + row;
            b_r[b][0] = *reinterpret_cast<const f4 *>(&sBm[buf][0][rb][8 * kk]);
            b_r[b][1] = *reinterpret_cast<const f4 *>(&sBm[buf][0][rb][8 * kk + 4]);
            b_i[b][0] = *reinterpret_cast<const f4 *>(&sBm[buf][1][rb][8 * kk]);
            b_i[b][1] = *reinterpret_cast<const f4 *>(&sBm[buf][1][rb][8 * kk + 4]);
        }
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
            float ys[2];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) ys[cb] = b_r[cb][s8 >> 2][s8 & 3] + b_i[cb][s8 >> 2][s8 & 3];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const float xr = a_r[b][s8 >> 2][s8 & 3], xi = a_i[b][s8 >> 2][s8 & 3];
                const float xs = xr + xi;
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    p1[b][cb] = MM<float>::mma(xr, b_r[cb][s8 >> 2][s8 & 3], p1[b][cb]);
                    p2[b][cb] = MM<float>::mma(xi, b_i[cb][s8 >> 2][s8 & 3], p2[b][cb]);
                    p3[b][cb] = MM<float>::mma(xs, ys[cb], p3[b][cb]);
                }
            }
        }
        }
        if (c + 1 < nch) store(buf ^ 1, next);
        __syncthreads();
    };
    FwdStage s0, s1;
    if (nch > 0) {
        load(0, s0);
        store(0, s0);
    }
    if (nch > 1) load(1, s1);
    __syncthreads();
    int c = 0;
    const int nwhole = ((N & 3) == 0) ? nch - 1 : 0;   // tiles 0 .. nch - 2 are whole
    for (; c + 4 <= nwhole; c += 2) {
        step(c, s1, s0, std::true_type());
        step(c + 1, s0, s1, std::true_type());
    }
    for (; c + 1 < nch; c += 2) {
        step(c, s1, s0, std::false_type());
        step(c + 1, s0, s1, std::false_type());
    }
    if (c < nch) step(c, s1, s0, std::false_type());
    float *pp = part + ((int64_t)split * P.nf + k) * P.mp * P.mp * 2;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int r = tr * 64 + 32 * wr + 16 * cb + row;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ee = te * 64 + 32 * we + 16 * b + MM<float>::out_row(kk, i);
                const int64_t o = ((int64_t)ee * P.mp + r) * 2;
                pp[o] = p1[b][cb][i] - p2[b][cb][i];
                pp[o + 1] = (p3[b][cb][i] - p1[b][cb][i]) - p2[b][cb][i];
            }
        }
    }
}

// Forward, FP32 tables with 16-byte aligned rows (N a multiple of 4).  The
// same tiles and waves as above, pixels consumed 16 at a time, and no
// staging registers: the tile rows of G_e and G_r (re, im) go from global
// memory straight into LDS (global_load_lds, 16 bytes per lane), double
// buffered, next to delta for the step's 16 pixels (as float, zero beyond
// N), and each wave scales its own B fragments by delta after reading them.
// Tile rows are 64 bytes, their four 16-byte chunks XOR-swizzled by
// (row / 2) mod 4 (a fragment read of 16 rows then meets no bank twice);
// a lane fills slot l mod 4 of row l / 4 and so loads the global chunk that
// the swizzle puts there.  Rows beyond m read row m - 1 and pixels beyond N
// read the row's last chunk: their outputs are never read, or delta is
// zero there.  With 32 KiB of LDS and about 100 registers a CU holds four
// workgroups; consecutive workgroups are the tiles of one pixel split
// on one XCD, which then reads each table row of the split from HBM about
// once.
constexpr int kFdKC = 16, kFdArr = 64 * 64, kFdBuf = 4 * kFdArr + 64;
constexpr int64_t kFdSplitPx = 16384;   // longest pixel split (1024 k-steps)
typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ int fd_off(int row, int ch) { return row * 64 + 16 * (ch ^ ((row >> 1) & 3)); }

// out[x] = (float)delta[x] for x < N, 0 for N <= x < n
__global__ void k_delta_cast(int64_t N, int64_t n, const double *__restrict__ delta, float *__restrict__ out) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) out[x] = x < N ? (float)delta[x] : 0.0f;
}

__global__ void __launch_bounds__(256, 4) k_forward_f32(FwdParams P, const float *__restrict__ Gr,
                                                        const float *__restrict__ Gi, const float *__restrict__ df,
                                                        float *__restrict__ part) {
    __shared__ __align__(16) unsigned char sm[2][kFdBuf];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kk = lane >> 4;
    const int we = wave >> 1, wr = wave & 1;
    int te, tr, split, k;
    fwd_block(P, te, tr, split, k);
    if (P.dmin >= 32 && max_circ_dist(P.m, te * 64, 64, tr * 64, 64) < P.dmin) return;
    const bool idle = fwd_block_idle(P, te, tr, we, wr);
    const int64_t N = P.N;
    const int64_t ks = (int64_t)split * P.kchunk;
    const int64_t ke = std::min<int64_t>(N, ks + P.kchunk);
    const int nch = (int)((ke - ks + kFdKC - 1) / kFdKC);
    // this lane's staging slot: tile row rl of each array, global chunk ch
    const int rl = 16 * wave + (lane >> 2);
    const int ch = (lane & 3) ^ ((rl >> 1) & 3);
    const int64_t go = (int64_t)k * P.m * N;
    const float *ae = Gr + go + (int64_t)std::min(te * 64 + rl, P.m - 1) * N;
    const float *ai = Gi + go + (int64_t)std::min(te * 64 + rl, P.m - 1) * N;
    const float *be = Gr + go + (int64_t)std::min(tr * 64 + rl, P.m - 1) * N;
    const float *bi = Gi + go + (int64_t)std::min(tr * 64 + rl, P.m - 1) * N;
    auto stage = [&](int c, int buf) {
        const int64_t xc = ks + (int64_t)c * kFdKC;
        const int64_t x = std::min<int64_t>(xc + 4 * ch, N - 4);
        unsigned char *d = sm[buf] + wave * 16 * 64;   // rows 16 wave .. 16 wave + 15
        __builtin_amdgcn_global_load_lds(ae + x, (lds_void_t *)d, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(ai + x, (lds_void_t *)(d + kFdArr), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(be + x, (lds_void_t *)(d + 2 * kFdArr), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(bi + x, (lds_void_t *)(d + 3 * kFdArr), 16, 0, 0);
        if (lane == 0)   // delta at pixels xc + 4 wave .. + 3
            __builtin_amdgcn_global_load_lds(df + xc + 4 * wave, (lds_void_t *)(sm[buf] + 4 * kFdArr + 16 * wave),
                                             16, 0, 0);
    };
    // (a + ib)(c + id) with three real products: P1 = ac, P2 = bd,
    // P3 = (a + b)(c + d); re = P1 - P2, im = P3 - P1 - P2
    f4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) p1[b][c] = p2[b][c] = p3[b][c] = f4{0, 0, 0, 0};
    if (nch > 0) stage(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) stage(c + 1, buf ^ 1);
        if (!idle) {
            const unsigned char *sb = sm[buf];
            f4 a_r[2], a_i[2], b_r[2], b_i[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int ra = 32 * we + 16 * b + row, rb = 32 * wr + 16 * b + row;
                a_r[b] = *reinterpret_cast<const f4 *>(sb + fd_off(ra, kk));
                a_i[b] = *reinterpret_cast<const f4 *>(sb + kFdArr + fd_off(ra, kk));
                b_r[b] = *reinterpret_cast<const f4 *>(sb + 2 * kFdArr + fd_off(rb, kk));
                b_i[b] = *reinterpret_cast<const f4 *>(sb + 3 * kFdArr + fd_off(rb, kk));
            }
            const f4 dl = *reinterpret_cast<const f4 *>(sb + 4 * kFdArr + 16 * kk);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                b_r[cb] *= dl;
                b_i[cb] *= dl;
            }
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                float ys[2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) ys[cb] = b_r[cb][s4] + b_i[cb][s4];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const float xr = a_r[b][s4], xi = a_i[b][s4];
                    const float xs = xr + xi;
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        p1[b][cb] = MM<float>::mma(xr, b_r[cb][s4], p1[b][cb]);
                        p2[b][cb] = MM<float>::mma(xi, b_i[cb][s4], p2[b][cb]);
                        p3[b][cb] = MM<float>::mma(xs, ys[cb], p3[b][cb]);
                    }
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);   // tile c + 1 has landed in LDS
        __syncthreads();
    }
    if (idle) return;
    float *pp = part + ((int64_t)split * P.nf + k) * P.mp * P.mp * 2;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int r = tr * 64 + 32 * wr + 16 * cb + row;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ee = te * 64 + 32 * we + 16 * b + MM<float>::out_row(kk, i);
                const int64_t o = ((int64_t)ee * P.mp + r) * 2;
                pp[o] = p1[b][cb][i] - p2[b][cb][i];
                pp[o + 1] = (p3[b][cb][i] - p1[b][cb][i]) - p2[b][cb][i];
            }
        }
    }
}

// ------------------------------------------------------------------ 16-bit, LDS-staged
// Forward with 16-bit tables on the 16x16x32 matrix cores (FP32
// accumulation), tiled as the FP32 kernel: a 64 x 64 (e, r) tile per
// workgroup, waves 2 x 2 of 32 x 32, 32 pixels per k-step.  Both operands
// take eight consecutive pixels of one row per lane, which the tables store
// contiguously, so a thread stages eight pixels of one row of G_e and of
// G_r delta (delta pre-scaled to float) with 16-byte loads, and a fragment
// is one 16-byte LDS read.  The four 16-byte chunks of a 64-byte tile row
// are XOR-swizzled by (row / 2) mod 4, which puts the reads of a fragment
// on distinct banks.  Tiles are double buffered.
constexpr int kF16KC = 32, kF16Arr = 64 * kF16KC * 2;   // one array of a tile (bytes)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int f16_off(int row, int ch) { return row * 64 + 16 * (ch ^ ((row >> 1) & 3)); }

// out[x] = delta[x] / max |delta| as float (0 if delta is zero)
__global__ void k_delta_f32(int64_t N, const double *__restrict__ delta, const double *__restrict__ dmax,
                            float *__restrict__ out) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    const double inv = dmax[0] > 0.0 ? 1.0 / dmax[0] : 0.0;
    out[x] = (float)(delta[x] * inv);
}

struct F16Stage {
    u32x4 ar, ai, br, bi;
    f4 d0, d1;
};

__device__ __forceinline__ void f16_stage_load(const unsigned short *__restrict__ gr,
                                               const unsigned short *__restrict__ gi,
                                               const float *__restrict__ df, int m, int64_t N, int e_row,
                                               int r_row, int64_t xs, int64_t ke, bool vec, F16Stage &v) {
    const u32x4 z = {0u, 0u, 0u, 0u};
    if (vec) {
        v.ar = e_row < m ? *reinterpret_cast<const u32x4 *>(gr + (int64_t)e_row * N + xs) : z;
        v.ai = e_row < m ? *reinterpret_cast<const u32x4 *>(gi + (int64_t)e_row * N + xs) : z;
        v.br = r_row < m ? *reinterpret_cast<const u32x4 *>(gr + (int64_t)r_row * N + xs) : z;
        v.bi = r_row < m ? *reinterpret_cast<const u32x4 *>(gi + (int64_t)r_row * N + xs) : z;
        v.d0 = *reinterpret_cast<const f4 *>(df + xs);
        v.d1 = *reinterpret_cast<const f4 *>(df + xs + 4);
    } else {
        unsigned short a_r[8], a_i[8], b_r[8], b_i[8];
        float d[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t x = xs + q;
            const bool okx = x < ke;
            const bool oka = okx && e_row < m, okb = okx && r_row < m;
            a_r[q] = oka ? gr[(int64_t)e_row * N + x] : (unsigned short)0;
            a_i[q] = oka ? gi[(int64_t)e_row * N + x] : (unsigned short)0;
            b_r[q] = okb ? gr[(int64_t)r_row * N + x] : (unsigned short)0;
            b_i[q] = okb ? gi[(int64_t)r_row * N + x] : (unsigned short)0;
            d[q] = okx ? df[x] : 0.0f;
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            v.ar[h] = a_r[2 * h] | ((unsigned)a_r[2 * h + 1] << 16);
            v.ai[h] = a_i[2 * h] | ((unsigned)a_i[2 * h + 1] << 16);
            v.br[h] = b_r[2 * h] | ((unsigned)b_r[2 * h + 1] << 16);
            v.bi[h] = b_i[2 * h] | ((unsigned)b_i[2 * h + 1] << 16);
        }
        v.d0 = f4{d[0], d[1], d[2], d[3]};
        v.d1 = f4{d[4], d[5], d[6], d[7]};
    }
}

// eight 16-bit values times delta, rounded back to the storage type
template <typename S, typename V>
__device__ __forceinline__ u32x4 f16_scale(u32x4 raw, f4 d0, f4 d1) {
    const V v = __builtin_bit_cast(V, raw);
    V o;
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = MM16<S>::from_f((float)v[i] * (i < 4 ? d0[i] : d1[i - 4]));
    return __builtin_bit_cast(u32x4, o);
}

template <typename S>
__global__ void __launch_bounds__(256, 2) k_forward16_lds(FwdParams P, const S *__restrict__ Gr,
                                                          const S *__restrict__ Gi, const float *__restrict__ df,
                                                          float *__restrict__ part) {
    using V = typename MM16<S>::vec;
    __shared__ __align__(16) unsigned char sA[2][2 * kF16Arr];   // [buffer][re, im] G_e rows
    __shared__ __align__(16) unsigned char sB[2][2 * kF16Arr];   // [buffer][re, im] G_r delta rows
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kk = lane >> 4;
    const int we = wave >> 1, wr = wave & 1;
    int te, tr, split, k;
    fwd_block(P, te, tr, split, k);
    const int64_t N = P.N;
    const unsigned short *gr = reinterpret_cast<const unsigned short *>(Gr + (int64_t)k * P.m * N);
    const unsigned short *gi = reinterpret_cast<const unsigned short *>(Gi + (int64_t)k * P.m * N);
    const int64_t ks = (int64_t)split * P.kchunk;
    const int64_t ke = std::min<int64_t>(N, ks + P.kchunk);
    const int nch = (int)((ke - ks + kF16KC - 1) / kF16KC);
    const int srow = tid >> 2, sch = tid & 3;
    const int e_row = te * 64 + srow, r_row = tr * 64 + srow;
    const int so = f16_off(srow, sch);
    // waves whose block is never used only stage (see k_forward_f32)
    if (P.dmin >= 32 && max_circ_dist(P.m, te * 64, 64, tr * 64, 64) < P.dmin) return;
    const bool idle = fwd_block_idle(P, te, tr, we, wr);
    f4 re[2][2], im[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) re[b][c] = im[b][c] = f4{0, 0, 0, 0};
    auto vec_ok = [&](int64_t xc) { return ((N & 7) == 0) && (xc + kF16KC <= ke); };
    auto load = [&](int c, F16Stage &v) {
        const int64_t xc = ks + (int64_t)c * kF16KC;
        f16_stage_load(gr, gi, df, P.m, N, e_row, r_row, xc + 8 * sch, ke, vec_ok(xc), v);
    };
    auto store = [&](int buf, const F16Stage &v) {
        *reinterpret_cast<u32x4 *>(sA[buf] + so) = v.ar;
        *reinterpret_cast<u32x4 *>(sA[buf] + kF16Arr + so) = v.ai;
        *reinterpret_cast<u32x4 *>(sB[buf] + so) = f16_scale<S, V>(v.br, v.d0, v.d1);
        *reinterpret_cast<u32x4 *>(sB[buf] + kF16Arr + so) = f16_scale<S, V>(v.bi, v.d0, v.d1);
    };
    // Tiles are loaded two steps ahead into two register sets used in turn:
    // step c computes on tile c (LDS), issues the loads of tile c + 2 and
    // stores tile c + 1, loaded a step earlier, to the other buffer.  Each
    // load then has two steps of MFMAs to arrive in.
    // FUT: tile c + 2 exists and is whole (16-byte loads, no tests), so the
    // steady state has unconditional loads and exact load-counter waits.
    auto step = [&](int c, F16Stage &next, F16Stage &fut, auto fut_tag) {
        const int buf = c & 1;
        if (decltype(fut_tag)::value)
            f16_stage_load(gr, gi, df, P.m, N, e_row, r_row, ks + (int64_t)(c + 2) * kF16KC + 8 * sch, ke, true,
                           fut);
        else if (c + 2 < nch)
            load(c + 2, fut);
        if (!idle) {
            V a_r[2], a_i[2], a_n[2], b_r[2], b_i[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int ra = 32 * we + 16 * b + row, rb = 32 * wr + 16 * b + row;
                a_r[b] = *reinterpret_cast<const V *>(sA[buf] + f16_off(ra, kk));
                a_i[b] = *reinterpret_cast<const V *>(sA[buf] + kF16Arr + f16_off(ra, kk));
                a_n[b] = neg(a_i[b]);
                b_r[b] = *reinterpret_cast<const V *>(sB[buf] + f16_off(rb, kk));
                b_i[b] = *reinterpret_cast<const V *>(sB[buf] + kF16Arr + f16_off(rb, kk));
            }
            // (ar + i ai)(br + i bi) = ar br - ai bi + i (ar bi + ai br)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    re[b][cb] = MM16<S>::mma(a_r[b], b_r[cb], re[b][cb]);
                    re[b][cb] = MM16<S>::mma(a_n[b], b_i[cb], re[b][cb]);
                    im[b][cb] = MM16<S>::mma(a_r[b], b_i[cb], im[b][cb]);
                    im[b][cb] = MM16<S>::mma(a_i[b], b_r[cb], im[b][cb]);
                }
        }
        if (c + 1 < nch) store(buf ^ 1, next);
        __syncthreads();
    };
    F16Stage s0, s1;
    if (nch > 0) {
        load(0, s0);
        store(0, s0);
    }
    if (nch > 1) load(1, s1);
    __syncthreads();
    int c = 0;
    // tiles 0 .. nch - 2 are whole; the last may be partial
    const int nwhole = ((N & 7) == 0) ? nch - 1 : 0;
    for (; c + 4 <= nwhole; c += 2) {
        step(c, s1, s0, std::true_type());       // tile c + 1 in s1, tile c + 2 into s0
        step(c + 1, s0, s1, std::true_type());   // tile c + 2 in s0, tile c + 3 into s1
    }
    for (; c + 1 < nch; c += 2) {
        step(c, s1, s0, std::false_type());
        step(c + 1, s0, s1, std::false_type());
    }
    if (c < nch) step(c, s1, s0, std::false_type());
    float *pp = part + ((int64_t)split * P.nf + k) * P.mp * P.mp * 2;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int r = tr * 64 + 32 * wr + 16 * cb + row;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ee = te * 64 + 32 * we + 16 * b + 4 * kk + i;
                const int64_t o = ((int64_t)ee * P.mp + r) * 2;
                pp[o] = re[b][cb][i];
                pp[o + 1] = im[b][cb][i];
            }
        }
    }
}

// ------------------------------------------------------------------ 16-bit, large rings
// For large rings the 64 x 64 tiles above move 16 KB per 64 MFMAs and are
// bound by memory traffic.  This kernel takes 128 x 128 (e, r) tiles, waves 2 x 2
// of 64 x 64 (4 x 4 blocks of 16 x 16, 64 MFMAs per wave and step), which
// halves the bytes per MFMA.  The accumulators leave no registers for staged
// tiles, so both operands go from memory straight into LDS (16-byte direct
// loads, the chunk swizzle of the 64-tile kernel) from two plain tables: G
// for the e side and a copy of G times delta (rounded to the storage type
// as the 64-tile kernel rounds it) for the r side, whose rows are padded
// with zeros to a multiple of 32 pixels.  Rows at or beyond m read row m - 1
// (their outputs are dropped); on the e side a chunk beyond N reads the last
// whole chunk, which the zero padding on the r side multiplies by 0.
// It pays from m = 1024 (68 -> 36 ms for four frequencies on 1100^2 pixels,
// the table pass included); at m = 512 the table pass outweighed the gain
// (10.1 against 8.2 ms, measured before the table pass used 16-byte loads).
#ifndef RB_FWD16_BIG_M
#define RB_FWD16_BIG_M 1024
#endif
constexpr int kF16BigM = RB_FWD16_BIG_M;
constexpr int kFBT = 128;
constexpr int kFBArr = kFBT * kF16KC * 2;   // one array of a tile (bytes)

// Gd[k][r][x] = G[k][r][x] * df[x] (rows padded to np pixels with zeros);
// one thread per eight pixels of a row.
template <typename S>
__global__ void k_scale16(int64_t N, int64_t np, int64_t rows, const S *__restrict__ Gr,
                          const S *__restrict__ Gi, const float *__restrict__ df, S *__restrict__ Dr,
                          S *__restrict__ Di) {
    using V = typename MM16<S>::vec;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = np / 8;
    if (t >= rows * per) return;
    const int64_t row = t / per, x0 = (t - row * per) * 8;
    V vr, vi;
    if (x0 + 8 <= N) {
        // whole run: 16-byte loads (N is a multiple of 8 here, so rows and
        // runs are 16-byte aligned)
        const V gr = *reinterpret_cast<const V *>(Gr + row * N + x0);
        const V gi = *reinterpret_cast<const V *>(Gi + row * N + x0);
        const f4 d0 = *reinterpret_cast<const f4 *>(df + x0), d1 = *reinterpret_cast<const f4 *>(df + x0 + 4);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float d = q < 4 ? d0[q] : d1[q - 4];
            vr[q] = MM16<S>::from_f((float)gr[q] * d);
            vi[q] = MM16<S>::from_f((float)gi[q] * d);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t x = x0 + q;
            const bool ok = x < N;
            const float d = ok ? df[x] : 0.0f;
            const float gr = ok ? MM16<S>::to_f(Gr[row * N + x]) : 0.0f;
            const float gi = ok ? MM16<S>::to_f(Gi[row * N + x]) : 0.0f;
            vr[q] = MM16<S>::from_f(gr * d);
            vi[q] = MM16<S>::from_f(gi * d);
        }
    }
    *reinterpret_cast<V *>(Dr + row * np + x0) = vr;
    *reinterpret_cast<V *>(Di + row * np + x0) = vi;
}

// Stage one k-step (32 pixels from xc) of rows r0 .. r0 + 127 of a table
// with row stride `ld` into one LDS array: wave w fills rows 32 w .. 32 w +
// 31, sixteen rows per instruction; lane l writes chunk slot l % 4 of row
// l / 4 and so loads the chunk the swizzle puts there.
__device__ __forceinline__ void fb_stage(const unsigned short *__restrict__ g, int64_t ld, int m, int r0,
                                         int64_t xc, int64_t xmax, unsigned char *dst) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int rb = 32 * wave + 16 * i;
        const int rl = rb + (lane >> 2);
        const int r = min(r0 + rl, m - 1);
        const int ch = (lane & 3) ^ ((rl >> 1) & 3);
        const int64_t x = min(xc + 8 * ch, xmax);
        __builtin_amdgcn_global_load_lds(g + (int64_t)r * ld + x, (lds_void_t *)(dst + rb * 64), 16, 0, 0);
    }
}

template <typename S>
__global__ void __launch_bounds__(256, 2) k_forward16_big(FwdParams P, const S *__restrict__ Gr,
                                                          const S *__restrict__ Gi, const S *__restrict__ Dr,
                                                          const S *__restrict__ Di, int64_t np,
                                                          float *__restrict__ part) {
    using V = typename MM16<S>::vec;
    __shared__ __align__(16) unsigned char sA[2][2 * kFBArr];   // [buffer][re, im] G_e rows
    __shared__ __align__(16) unsigned char sB[2][2 * kFBArr];   // [buffer][re, im] G_r delta rows
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kk = lane >> 4;
    const int we = wave >> 1, wr = wave & 1;
    int te, tr, split, k;
    fwd_block(P, te, tr, split, k);
    if (P.dmin >= 32 && max_circ_dist(P.m, te * kFBT, kFBT, tr * kFBT, kFBT) < P.dmin) return;
    const bool idle = (te == tr && we > wr) ||
                      (P.dmin >= 32 && max_circ_dist(P.m, te * kFBT + 64 * we, 64, tr * kFBT + 64 * wr, 64) < P.dmin);
    const int64_t N = P.N;
    const unsigned short *ger = reinterpret_cast<const unsigned short *>(Gr + (int64_t)k * P.m * N);
    const unsigned short *gei = reinterpret_cast<const unsigned short *>(Gi + (int64_t)k * P.m * N);
    const unsigned short *gdr = reinterpret_cast<const unsigned short *>(Dr + (int64_t)k * P.m * np);
    const unsigned short *gdi = reinterpret_cast<const unsigned short *>(Di + (int64_t)k * P.m * np);
    const int64_t ks = (int64_t)split * P.kchunk;
    const int64_t ke = std::min<int64_t>(N, ks + P.kchunk);
    const int nch = (int)((ke - ks + kF16KC - 1) / kF16KC);
    auto stage = [&](int c, int buf) {
        const int64_t xc = ks + (int64_t)c * kF16KC;
        fb_stage(ger, N, P.m, te * kFBT, xc, N - 8, sA[buf]);
        fb_stage(gei, N, P.m, te * kFBT, xc, N - 8, sA[buf] + kFBArr);
        fb_stage(gdr, np, P.m, tr * kFBT, xc, np - 8, sB[buf]);
        fb_stage(gdi, np, P.m, tr * kFBT, xc, np - 8, sB[buf] + kFBArr);
    };
    f4 re[4][4], im[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) re[b][c] = im[b][c] = f4{0, 0, 0, 0};
    if (nch > 0) stage(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) stage(c + 1, buf ^ 1);
        if (!idle) {
            V b_r[4], b_i[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int rb = 64 * wr + 16 * cb + row;
                b_r[cb] = *reinterpret_cast<const V *>(sB[buf] + f16_off(rb, kk));
                b_i[cb] = *reinterpret_cast<const V *>(sB[buf] + kFBArr + f16_off(rb, kk));
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int ra = 64 * we + 16 * b + row;
                const V a_r = *reinterpret_cast<const V *>(sA[buf] + f16_off(ra, kk));
                const V a_i = *reinterpret_cast<const V *>(sA[buf] + kFBArr + f16_off(ra, kk));
                const V a_n = neg(a_i);
                // (ar + i ai)(br + i bi) = ar br - ai bi + i (ar bi + ai br)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    re[b][cb] = MM16<S>::mma(a_r, b_r[cb], re[b][cb]);
                    re[b][cb] = MM16<S>::mma(a_n, b_i[cb], re[b][cb]);
                    im[b][cb] = MM16<S>::mma(a_r, b_i[cb], im[b][cb]);
                    im[b][cb] = MM16<S>::mma(a_i, b_r[cb], im[b][cb]);
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);   // tile c + 1 has landed in LDS
        __syncthreads();
    }
    if (idle) return;
    float *pp = part + ((int64_t)split * P.nf + k) * P.mp * P.mp * 2;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int r = tr * kFBT + 64 * wr + 16 * cb + row;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ee = te * kFBT + 64 * we + 16 * b + 4 * kk + i;
                const int64_t o = ((int64_t)ee * P.mp + r) * 2;
                pp[o] = re[b][cb][i];
                pp[o + 1] = im[b][cb][i];
            }
        }
    }
}

}  // namespace

// ---------------------------------------------------------------- host side
// Compute units of the current device (256 on MI355X), queried on every
// call: the library keeps no mutable state between calls.
static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

// The 128 x 128-tile 16-bit kernel: large rings, rows of whole 16-byte chunks.
static bool fwd16_big(const rb_geometry *g, rb_dtype dt) {
    const int64_t N = (int64_t)g->nx * g->ny;
    return (dt == RB_BF16 || dt == RB_F16) && g->m >= kF16BigM && N % 8 == 0;
}

// The FP32 kernel with direct loads: rows of whole 16-byte chunks.
static bool fwd32_direct(const rb_geometry *g, rb_dtype dt) {
    return dt == RB_F32 && ((int64_t)g->nx * g->ny) % 4 == 0;
}

static FwdParams fwd_params(const rb_geometry *g, const double *freqs, int nf, rb_dtype dt) {
    FwdParams P;
    const int tile = fwd16_big(g, dt) ? kFBT : 64;
    P.m = g->m;
    P.mp = (g->m + tile - 1) / tile * tile;
    P.N = (int64_t)g->nx * g->ny;
    P.nf = nf;
    P.ntl = P.mp / tile;
    const int ntri = P.ntl * (P.ntl + 1) / 2;
    // about four rounds of resident workgroups (two per CU, four for the
    // FP32 kernel with direct loads), rounded down so the last round is full
    const int want = 4 * (fwd32_direct(g, dt) ? 4 : 2) * device_cus();
    int nsplit = std::max(1, want / (ntri * nf));
    // the kernels with direct loads (FP32, and 16-bit for large rings) also
    // keep a split to at most kFdSplitPx pixels: the tiles of a split share
    // its table rows in L2 only while they stay within a few k-steps of each
    // other, and long workgroups drift apart (FP32, 1024 elements / 1100^2:
    // 7 splits 144.4 ms, 30 splits 138.1 ms, 60 splits 135.0 ms for the
    // public call)
    if (fwd32_direct(g, dt) || fwd16_big(g, dt))
        nsplit = std::max<int64_t>(nsplit, (P.N + kFdSplitPx - 1) / kFdSplitPx);
    const int kq = (dt == RB_BF16 || dt == RB_F16) ? 32 : 16;
    int64_t kchunk = (P.N + nsplit - 1) / nsplit;
    kchunk = (kchunk + kq - 1) / kq * kq;
    if (kchunk < kq) kchunk = kq;
    nsplit = (int)((P.N + kchunk - 1) / kchunk);
    P.nsplit = nsplit;
    P.kchunk = kchunk;
    P.ntri = ntri;
    P.dmin = 0;
    const double dA = g->h * g->h;
    for (int k = 0; k < nf; ++k) {
        const double om = 2.0 * M_PI * (freqs ? freqs[k] : 1.0);
        P.cg[k] = om * om * dA;
    }
    return P;
}

// workspace: max |delta|, the split partials, (16-bit) delta as float, and
// (large rings) the G delta tables with rows padded to np pixels
struct FwdWs {
    double *dmax, *dparts;
    void *part;
    float *df;
    void *dr, *di;
    int64_t np;
};

static FwdWs carve_fwd(Carver &c, const FwdParams &P, rb_dtype dt, bool big) {
    const size_t es = dt == RB_F64 ? 8 : 4;
    FwdWs w;
    w.dmax = c.take<double>(1);
    w.dparts = (dt == RB_BF16 || dt == RB_F16) ? c.take<double>(kReduceBlocks) : nullptr;
    w.part = c.take<char>((size_t)P.nsplit * P.nf * P.mp * P.mp * 2 * es);
    w.df = (dt == RB_BF16 || dt == RB_F16 || (dt == RB_F32 && P.N % 4 == 0)) ? c.take<float>((size_t)P.N + 16)
                                                                               : nullptr;
    w.np = (P.N + kF16KC - 1) / kF16KC * kF16KC;
    w.dr = big ? (void *)c.take<uint16_t>((size_t)P.nf * P.m * w.np) : nullptr;
    w.di = big ? (void *)c.take<uint16_t>((size_t)P.nf * P.m * w.np) : nullptr;
    return w;
}

size_t forward_workspace_bytes(const rb_geometry *g, int nf, rb_dtype dt) {
    FwdParams P = fwd_params(g, nullptr, nf, dt);
    Carver c(nullptr, 0);
    carve_fwd(c, P, dt, fwd16_big(g, dt));
    return c.used + 256;
}

rb_status forward_impl(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                       rb_dtype dt, const double *freqs, int nf, const double *delta, double *d_out, void *ws,
                       size_t ws_bytes, hipStream_t st, int dmin) {
    if (ws_bytes < forward_workspace_bytes(g, nf, dt)) {
        set_error("forward workspace too small: need %zu bytes", forward_workspace_bytes(g, nf, dt));
        return RB_ENOMEM;
    }
    FwdParams P = fwd_params(g, freqs, nf, dt);
    P.dmin = dmin;
    const bool big = fwd16_big(g, dt);
    Carver c(ws, ws_bytes);
    FwdWs w = carve_fwd(c, P, dt, big);
    const unsigned nblk = (unsigned)((int64_t)P.ntri * P.nsplit * nf);
    const int64_t tot = (int64_t)nf * P.m * P.m;
    switch (dt) {
        case RB_F64: {
            dim3 grid(P.ntri, P.nsplit, nf);
            k_forward<double><<<grid, 256, 0, st>>>(P, (const double *)G_re, (const double *)G_im, delta,
                                                    (double *)w.part);
            RB_LAUNCHED();
            k_forward_reduce<double><<<blocks_for(tot, 256), 256, 0, st>>>(P, (const double *)w.part, nullptr,
                                                                           nullptr, d_out);
            break;
        }
        case RB_F32:
            if (fwd32_direct(g, dt)) {
                k_delta_cast<<<blocks_for(P.N + 16, 256), 256, 0, st>>>(P.N, P.N + 16, delta, w.df);
                RB_LAUNCHED();
                k_forward_f32<<<nblk, 256, 0, st>>>(P, (const float *)G_re, (const float *)G_im, w.df,
                                                    (float *)w.part);
            } else {
                k_forward_f32_regs<<<dim3(P.ntri, P.nsplit, nf), 256, 0, st>>>(P, (const float *)G_re,
                                                                               (const float *)G_im, delta,
                                                                               (float *)w.part);
            }
            RB_LAUNCHED();
            k_forward_reduce<float><<<blocks_for(tot, 256), 256, 0, st>>>(P, (const float *)w.part, gscale,
                                                                          nullptr, d_out);
            break;
        case RB_BF16:
        case RB_F16:
            RB_TRY(reduce_absmax_f64(delta, P.N, w.dparts, w.dmax, st));
            k_delta_f32<<<blocks_for(P.N, 256), 256, 0, st>>>(P.N, delta, w.dmax, w.df);
            RB_LAUNCHED();
            if (big) {
                const int64_t rows = (int64_t)nf * P.m;
                auto go = [&](auto tag) {
                    using S = decltype(tag);
                    k_scale16<S><<<blocks_for(rows * (w.np / 8), 256), 256, 0, st>>>(
                        P.N, w.np, rows, (const S *)G_re, (const S *)G_im, w.df, (S *)w.dr, (S *)w.di);
                    RB_LAUNCHED();
                    k_forward16_big<S><<<nblk, 256, 0, st>>>(P, (const S *)G_re, (const S *)G_im,
                                                             (const S *)w.dr, (const S *)w.di, w.np,
                                                             (float *)w.part);
                    return RB_OK;
                };
                if (dt == RB_BF16)
                    RB_TRY(go(__hip_bfloat16()));
                else
                    RB_TRY(go(__half()));
            } else if (dt == RB_BF16)
                k_forward16_lds<__hip_bfloat16><<<nblk, 256, 0, st>>>(P, (const __hip_bfloat16 *)G_re,
                                                                      (const __hip_bfloat16 *)G_im, w.df,
                                                                      (float *)w.part);
            else
                k_forward16_lds<__half><<<nblk, 256, 0, st>>>(P, (const __half *)G_re, (const __half *)G_im,
                                                              w.df, (float *)w.part);
            RB_LAUNCHED();
            k_forward_reduce<float><<<blocks_for(tot, 256), 256, 0, st>>>(P, (const float *)w.part, gscale,
                                                                          w.dmax, d_out);
            break;
    }
    RB_LAUNCHED();
    return RB_OK;
}

rb_status check_contraction(const rb_geometry *g, const void *G_re, const void *G_im, const float *scale,
                                   rb_dtype dt, const double *freqs, int32_t nf) {
    RB_TRY(check_geometry(g));
    RB_TRY(check_freqs(freqs, nf));
    RB_CHECK_ARG(dt >= RB_F64 && dt <= RB_F16, "unknown dtype %d", (int)dt);
    RB_CHECK_ARG(G_re && G_im, "G_re/G_im are NULL");
    RB_CHECK_ARG(((uintptr_t)G_re & 15) == 0 && ((uintptr_t)G_im & 15) == 0,
                 "G_re/G_im must be 16-byte aligned (the kernels read rows in 16-byte pieces)");
    RB_CHECK_ARG(!(dt == RB_BF16 || dt == RB_F16) || scale, "scale is required for 16-bit storage");
    return RB_OK;
}

}  // namespace rb

extern "C" {

size_t rb_forward_workspace_bytes(const rb_geometry *g, int32_t nf, rb_dtype dtype) {
    if (rb::check_geometry(g) != RB_OK || nf < 1 || nf > RB_MAX_NF) return 0;
    return rb::forward_workspace_bytes(g, nf, dtype);
}

rb_status rb_born_forward(const rb_geometry *g, const void *G_re, const void *G_im, const float *scale,
                          rb_dtype dtype, const double *freqs_hz, int32_t nf, const double *delta, double *d_out,
                          void *ws, size_t ws_bytes, void *stream) {
    rb::clear_error();
    RB_TRY(rb::check_contraction(g, G_re, G_im, scale, dtype, freqs_hz, nf));
    RB_CHECK_ARG(delta && d_out, "delta/d_out are NULL");
    RB_CHECK_ARG(ws, "workspace is NULL");
    return rb::forward_impl(g, G_re, G_im, scale, dtype, freqs_hz, nf, delta, d_out, ws, ws_bytes,
                            rb::as_stream(stream));
}

}  // extern "C"
