// Weighted adjoint (backprojection) of the Born operator with the diagonal of
// the Gauss-Newton Hessian (paper, Inverse Problem section, Eqs. 8-10;
// linearisation of Eq. 1 in q = 1/c^2 with Green's functions from Eqs. 4-5).
//
//   grad(x) = omega^2 h^2 Re sum_e conj(G_e(x)) Y_e(x),
//   Y_e(x)  = sum_r A_er conj(G_r(x)),      A = W . D
//   hd(x)   = omega^4 h^4 sum_e |G_e(x)|^2 Z_e(x),
//   Z_e(x)  = sum_r W_er |G_r(x)|^2
//
// A dense contraction over emitter x receiver pairs, so it runs on the matrix
// cores.  The complex product is expanded into real MFMAs and the reduction
// over e against G_e(x) is fused into the epilogue, so Y and Z never leave
// registers.  A k-permutation (lane group kk supplies k = 4 kk + s at MFMA
// step s) lets each lane fetch its A fragment with one vector load.  Blocks
// of A whose weights are all zero (the receiver selection removes a band
// around the diagonal) are skipped per 16x16 block.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "born.h"
#include "common.h"
#include "mma.h"

namespace rb {
namespace {

// ------------------------------------------------------------------ adjoint
// WG = 4 waves; wave w owns 16*CB pixels; rows are processed 16*RB at a time.
template <typename T, int RB, int CB>
__global__ void __launch_bounds__(256) k_adjoint(AdjParams P, const T *__restrict__ Gr, const T *__restrict__ Gi,
                                                 const T *__restrict__ Ar, const T *__restrict__ Ai,
                                                 const T *__restrict__ Wt, const uint8_t *__restrict__ flags,
                                                 double *__restrict__ grad, double *__restrict__ hd) {
    using acc_t = typename MM<T>::acc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kk = lane >> 4;
    const int64_t N = P.N;
    const int64_t xw = (int64_t)blockIdx.x * (64 * CB) + (int64_t)wave * 16 * CB;
    double gacc[CB], hacc[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) gacc[c] = hacc[c] = 0.0;

    for (int k = 0; k < P.nf; ++k) {
        const T *gr = Gr + (int64_t)k * P.m * N;
        const T *gi = Gi + (int64_t)k * P.m * N;
        const T *ar = Ar + (int64_t)k * P.mp * P.mp;
        const T *ai = Ai + (int64_t)k * P.mp * P.mp;
        const T *wt = Wt + (int64_t)k * P.mp * P.mp;
        const uint8_t *fl = flags + (int64_t)k * P.nb * P.nb;
        T gp[CB], hp[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) gp[c] = hp[c] = T(0);
        for (int ec = 0; ec < P.mp; ec += 16 * RB) {
            acc_t yr[RB][CB], yn[RB][CB], z[RB][CB];
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int c = 0; c < CB; ++c) yr[b][c] = yn[b][c] = z[b][c] = acc_t{0, 0, 0, 0};
            for (int rc = 0; rc < P.mp; rc += 16) {
                bool on[RB];
                bool any = false;
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    const int eb = ec / 16 + b;
                    on[b] = (eb < P.nb) && fl[eb * P.nb + rc / 16];
                    any |= on[b];
                }
                if (!any) continue;
                T br[4][CB], bi[4][CB], b2[4][CB];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int r = rc + 4 * kk + s;
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        const int64_t x = xw + 16 * c + row;
                        const bool ok = (r < P.m) && (x < N);
                        br[s][c] = ld(gr + (int64_t)r * N + x, ok);
                        bi[s][c] = ld(gi + (int64_t)r * N + x, ok);
                        b2[s][c] = br[s][c] * br[s][c] + bi[s][c] * bi[s][c];
                    }
                }
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    if (!on[b]) continue;
                    const int64_t off = (int64_t)(ec + 16 * b + row) * P.mp + rc + 4 * kk;
                    T va[4], vi[4], vw[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        va[s] = ar[off + s];
                        vi[s] = ai[off + s];
                        vw[s] = wt[off + s];
                    }
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
#pragma unroll
                        for (int c = 0; c < CB; ++c) {
                            yr[b][c] = MM<T>::mma(va[s], br[s][c], yr[b][c]);
                            yr[b][c] = MM<T>::mma(vi[s], bi[s][c], yr[b][c]);
                            yn[b][c] = MM<T>::mma(va[s], bi[s][c], yn[b][c]);
                            yn[b][c] = MM<T>::mma(-vi[s], br[s][c], yn[b][c]);
                            z[b][c] = MM<T>::mma(vw[s], b2[s][c], z[b][c]);
                        }
                    }
                }
            }
            // fused epilogue: reduce over the e rows of this chunk against G_e
#pragma unroll
            for (int b = 0; b < RB; ++b) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = ec + 16 * b + MM<T>::out_row(kk, i);
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        const int64_t x = xw + 16 * c + row;
                        const bool ok = (e < P.m) && (x < N);
                        const T ge_r = ld(gr + (int64_t)e * N + x, ok);
                        const T ge_i = ld(gi + (int64_t)e * N + x, ok);
                        gp[c] += ge_r * yr[b][c][i] - ge_i * yn[b][c][i];
                        hp[c] += (ge_r * ge_r + ge_i * ge_i) * z[b][c][i];
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            gacc[c] += (double)gp[c] * P.cg[k];
            hacc[c] += (double)hp[c] * P.ch[k];
        }
    }
    // sum the four lane groups that hold the same pixel (fixed order)
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        double g = gacc[c], h = hacc[c];
        g += __shfl_xor(g, 16);
        h += __shfl_xor(h, 16);
        g += __shfl_xor(g, 32);
        h += __shfl_xor(h, 32);
        const int64_t x = xw + 16 * c + row;
        if (kk == 0 && x < N) {
            grad[x] += g;
            if (hd) hd[x] += h;
        }
    }
}

// Operands of the adjoint: A = W . D (re, im) and W in the storage type,
// padded to mp x mp with zeros.  For 16-bit types A is divided by ascale[k]
// = max |W D| (1 if that is 0; W is 0/1-valued in the inversion, stored
// unscaled).
template <typename T>
__device__ __forceinline__ T cvt(double v);
template <>
__device__ __forceinline__ double cvt<double>(double v) { return v; }
template <>
__device__ __forceinline__ float cvt<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ __hip_bfloat16 cvt<__hip_bfloat16>(double v) { return __float2bfloat16((float)v); }
template <>
__device__ __forceinline__ __half cvt<__half>(double v) { return __float2half((float)v); }

// PERMUTE: within every 32-column chunk, receiver 4 s + kk is stored at
// column 8 kk + s (the operand order of k_adjoint_f32).
template <typename T, bool SCALED, bool PERMUTE = false>
__global__ void k_adj_prep(int m, int mp, int nf, const double *__restrict__ d, const double *__restrict__ w,
                           const float *__restrict__ ascale, T *__restrict__ Ar, T *__restrict__ Ai,
                           T *__restrict__ Wt) {
    const int64_t per = (int64_t)mp * mp;
    const int64_t tot = per * nf;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(idx / per);
        const int64_t rem = idx - (int64_t)k * per;
        const int e = (int)(rem / mp), r = (int)(rem - (int64_t)e * mp);
        double re = 0.0, im = 0.0, wv = 0.0;
        if (e < m && r < m) {
            const int64_t q = ((int64_t)k * m + e) * m + r;
            wv = w[q];
            re = wv * d[2 * q];
            im = wv * d[2 * q + 1];
            if (SCALED) {
                const float a = ascale[k];   // 0 when every weight is zero
                const double inv = a > 0.0f ? 1.0 / (double)a : 1.0;
                re *= inv;
                im *= inv;
            }
        }
        int64_t o = idx;
        if (PERMUTE) {
            const int kr = r & 31;
            o = idx - kr + 8 * (kr & 3) + (kr >> 2);
        }
        Ar[o] = cvt<T>(re);
        Ai[o] = cvt<T>(im);
        Wt[o] = cvt<T>(wv);
    }
}

// One workgroup per 16x16 block (eb, rb) and frequency, one thread per
// entry: flags[k][eb][rb] = 1 if any weight of the block is nonzero, and
// for 16-bit operands (amax != null) the block's max |W D| (as float bits;
// max is order-independent) folded into amax[k], which starts at zero.
__global__ void __launch_bounds__(256) k_adj_blocks(int m, int nb, const double *__restrict__ d,
                                                    const double *__restrict__ w, uint8_t *__restrict__ flags,
                                                    unsigned *__restrict__ amax) {
    __shared__ float sm[4];
    const int k = blockIdx.y, eb = blockIdx.x / nb, rb = blockIdx.x - (blockIdx.x / nb) * nb;
    const int e = eb * 16 + (threadIdx.x >> 4), r = rb * 16 + (threadIdx.x & 15);
    double wv = 0.0, re = 0.0, im = 0.0;
    if (e < m && r < m) {
        const int64_t q = ((int64_t)k * m + e) * m + r;
        wv = w[q];
        if (amax) {
            re = wv * d[2 * q];
            im = wv * d[2 * q + 1];
        }
    }
    const int any = __syncthreads_or(wv != 0.0);
    if (threadIdx.x == 0) flags[((int64_t)k * nb + eb) * nb + rb] = any ? 1 : 0;
    if (!amax) return;
    float v = (float)fmax(fabs(re), fabs(im));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float b = fmaxf(fmaxf(sm[0], sm[1]), fmaxf(sm[2], sm[3]));
        if (b > 0.0f) atomicMax(amax + k, __float_as_uint(b));
    }
}

// ------------------------------------------------------------------ FP32, LDS-staged
// Backprojection.  The workgroup owns 64 pixels; its four waves are 2
// (emitter halves) x 2 (pixel halves), each computing 32 e x 32 px of Y per
// chunk of 64 emitters.  Receivers are consumed 32 at a time: the G tile
// [32 r][64 px] (re, im) goes from global memory straight into LDS
// (global_load_lds, 16 bytes per lane), double buffered, so staging costs
// no registers and overlaps the MFMAs of the previous chunk.  Rows are
// unpadded; the 16-byte chunks of row r are XOR-swizzled by (r & 3), which
// puts the four lane groups of a B-fragment read (rows 4 s + kk) on distinct
// banks.  A is stored k-permuted, so a lane's eight A values of a chunk are
// two float4 loads (served from L2: A is shared by every workgroup),
// prefetched one chunk ahead.
constexpr int kAdjNT = 64, kAdjKC = 32, kAdjTile = kAdjKC * 64;

typedef __attribute__((address_space(3))) void lds_void_t;

// LDS offset (floats) of (tile row r, pixel px) in a swizzled [32][64] tile
__device__ __forceinline__ int adj_off(int r, int px) {
    return r * 64 + ((((px >> 2) ^ ((r & 3) << 2))) << 2) + (px & 3);
}

// Aligned full tiles: wave w fills rows 8 w .. 8 w + 7 of both arrays, four
// rows per instruction.  Lane l of an instruction writes LDS chunk
// (row l / 16, chunk l % 16), so it loads the global chunk that the swizzle
// puts there.  Rows at or beyond m read row m - 1: their A entries are zero.
__device__ __forceinline__ void adj_stage_async(const float *__restrict__ gr, const float *__restrict__ gi, int m,
                                                int64_t N, int rc, int64_t x0, float *sT) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int r0 = wave * 8 + j * 4;
        const int rl = r0 + (lane >> 4);
        const int r = min(rc + rl, m - 1);
        const int gc = (lane & 15) ^ ((rl & 3) << 2);
        const int64_t go = (int64_t)r * N + x0 + 4 * gc;
        __builtin_amdgcn_global_load_lds(gr + go, (lds_void_t *)(sT + r0 * 64), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(gi + go, (lds_void_t *)(sT + kAdjTile + r0 * 64), 16, 0, 0);
    }
}

// Ragged or unaligned tiles: through registers, zero beyond m and N.
__device__ __forceinline__ void adj_stage_regs(const float *__restrict__ gr, const float *__restrict__ gi, int m,
                                               int64_t N, int rc, int64_t x0, float *sT) {
    const int t = threadIdx.x;
    const int rl = t >> 3, r = rc + rl, p0 = (t & 7) * 8;
    float vr[8], vi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t x = x0 + p0 + q;
        const bool ok = r < m && x < N;
        vr[q] = ok ? gr[(int64_t)r * N + x] : 0.0f;
        vi[q] = ok ? gi[(int64_t)r * N + x] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        sT[adj_off(rl, p0 + q)] = vr[q];
        sT[kAdjTile + adj_off(rl, p0 + q)] = vi[q];
    }
}

// NB row blocks starting at b0.  The complex product Y = A conj(G) uses
// three real products, P1 = Ar Gr, P2 = Ai Gi, P3 = (Ar + Ai)(Gr - Gi)
// (Ar + Ai formed in registers), so Yr = P1 + P2 and Yi = P3 - P1 + P2; with
// the Hessian term Z = W |G|^2 (HESS) that is four MFMAs per block and step,
// each on a different accumulator.
template <int NB, bool HESS>
__device__ __forceinline__ void adj_mma_steps(const f4 (&va)[2][2], const f4 (&vi)[2][2], const f4 (&vw)[2][2],
                                              const float *sBr, const float *sBi, int kk, const int (&coff)[2],
                                              f4 (&p1)[2][2], f4 (&p2)[2][2], f4 (&p3)[2][2], f4 (&z)[2][2],
                                              int b0) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        // B fragments for four steps at a time (one LDS wait per half chunk)
        float br[4][2], bi[4][2];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int o = (4 * (4 * half + q4) + kk) * 64 + coff[cb];
                br[q4][cb] = sBr[o];
                bi[q4][cb] = sBi[o];
            }
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) {
        const int s8 = 4 * half + q4;
        float b2[2], bd[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            if (HESS) b2[cb] = br[q4][cb] * br[q4][cb] + bi[q4][cb] * bi[q4][cb];
            bd[cb] = br[q4][cb] - bi[q4][cb];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int b = b0 + q;
            const float a_r = va[b][s8 >> 2][s8 & 3], a_i = vi[b][s8 >> 2][s8 & 3];
            const float a_s = a_r + a_i;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                p1[b][cb] = MM<float>::mma(a_r, br[q4][cb], p1[b][cb]);
                p2[b][cb] = MM<float>::mma(a_i, bi[q4][cb], p2[b][cb]);
                p3[b][cb] = MM<float>::mma(a_s, bd[cb], p3[b][cb]);
                if (HESS) z[b][cb] = MM<float>::mma(vw[b][s8 >> 2][s8 & 3], b2[cb], z[b][cb]);
            }
        }
    }
    }
}

// Where a workgroup's work lies: pixel tile loc.tile(), frequency loc.k().
// A launch over one problem reads them from the grid (blockIdx), a grouped
// launch from the problem table.
struct GridLoc {
    __device__ __forceinline__ int64_t tile() const { return blockIdx.x; }
    __device__ __forceinline__ int k() const { return blockIdx.y; }
    __device__ __forceinline__ int group() const { return 0; }
};
struct ItemLoc {
    int64_t t;
    int kf, q;
    __device__ __forceinline__ int64_t tile() const { return t; }
    __device__ __forceinline__ int k() const { return kf; }
    __device__ __forceinline__ int group() const { return q; }   // emitter-pass group
};

// Kernel argument of a launch over one problem: grid (pixel tiles, frequencies).
struct AdjOne {
    using Loc = GridLoc;
    static constexpr bool kSplit = false;   // one workgroup per (pixel tile, frequency)
    AdjItem item;
    __device__ __forceinline__ const AdjItem &locate(Loc &) const { return item; }
};

// Kernel argument of a launch over one problem whose emitter passes are
// split into item.npg groups: grid (pixel tiles x groups, frequencies), the
// groups of a tile adjacent in logical order and, through the XCD remap, on
// one XCD at about the same time, so that they share its G tiles in L2.
struct AdjOneSplit {
    using Loc = ItemLoc;
    static constexpr bool kSplit = true;
    AdjItem item;
    __device__ __forceinline__ const AdjItem &locate(Loc &loc) const {
        const int64_t l = xcd_remap(blockIdx.x, gridDim.x);
        loc.t = l / item.npg;
        loc.q = (int)(l - loc.t * item.npg);
        loc.kf = blockIdx.y;
        return item;
    }
};

// Kernel argument of a launch over several problems: which problem a flat
// workgroup id belongs to, and its (frequency, pixel tile, group) there.
// Workgroup-uniform.
struct AdjGroupArg {
    using Loc = ItemLoc;
    static constexpr bool kSplit = true;
    AdjGroup G;
    __device__ __forceinline__ const AdjItem &locate(Loc &loc) const {
        const int b = blockIdx.x;
        int j = 0;
        while (j + 1 < G.n && b >= G.item[j + 1].begin) ++j;
        const AdjItem &it = G.item[j];
        const int local = b - it.begin;
        const int per = it.ntiles * it.npg;
        loc.kf = local / per;
        const int rem = local - loc.kf * per;
        loc.t = rem / it.npg;
        loc.q = rem - (int)loc.t * it.npg;
        return it;
    }
};

// HESS = false computes the gradient only (three MFMAs per block and step);
// its registers allow three workgroups per CU (34 KB of LDS each).  The
// argument is one problem (AdjOne: grid = pixel tiles x frequencies) or a
// group of problems (AdjGroup: flat grid over every problem's work items).
template <bool HESS, typename A>
__global__ void __launch_bounds__(256, HESS ? 2 : 3) k_adjoint_f32(const A args) {
    typename A::Loc loc;
    const AdjItem &it = args.locate(loc);
    const AdjParams &P = it.P;
    const float *__restrict__ Gr = (const float *)it.Gr;
    const float *__restrict__ Gi = (const float *)it.Gi;
    const float *__restrict__ Ar = (const float *)it.Ar;
    const float *__restrict__ Ai = (const float *)it.Ai;
    const float *__restrict__ Wt = (const float *)it.Wt;
    const uint8_t *__restrict__ flags = it.flags;
    double *__restrict__ pg = it.pg;
    double *__restrict__ ph = it.ph;
    __shared__ __align__(16) float sB[2][2 * kAdjTile];   // [buffer][re tile, im tile]
    __shared__ double sred[2][2][kAdjNT];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const int row = lane & 15, kk = lane >> 4;
    const int we = wave >> 1, wp = wave & 1;
    const int64_t N = P.N;
    const int64_t x0 = (int64_t)loc.tile() * kAdjNT;
    const bool vec = ((N & 3) == 0) && (x0 + kAdjNT <= N);   // workgroup-uniform
    // this lane's column offsets in the swizzled tile (rows 4 s + kk)
    int coff[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) coff[cb] = adj_off(kk, 32 * wp + 16 * cb + row) - kk * 64;
    const int nch = P.mp / kAdjKC;
    double gacc[2] = {0.0, 0.0}, hacc[2] = {0.0, 0.0};
    // this workgroup's emitter passes (64 emitters each): group qg of npg
    const int npg = A::kSplit ? it.npg : 1, qg = A::kSplit ? loc.group() : 0;
    const int npass = P.mp / 64 + ((P.mp & 63) ? 1 : 0);
    const int pass0 = A::kSplit ? qg * npass / npg : 0, pass1 = A::kSplit ? (qg + 1) * npass / npg : npass;

    {
        const int k = loc.k();   // one frequency per workgroup (finer work units)
        const float *gr = Gr + (int64_t)k * P.m * N;
        const float *gi = Gi + (int64_t)k * P.m * N;
        const float *ar = Ar + (int64_t)k * P.mp * P.mp;
        const float *ai = Ai + (int64_t)k * P.mp * P.mp;
        const float *wt = Wt + (int64_t)k * P.mp * P.mp;
        const uint8_t *fl = flags + (int64_t)k * P.nb * P.nb;
        float gp[2] = {0.0f, 0.0f}, hp[2] = {0.0f, 0.0f};
        for (int ec = 64 * pass0; ec < 64 * pass1; ec += 64) {
            f4 p1[2][2], p2[2][2], p3[2][2], z[2][2];
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) p1[b][c] = p2[b][c] = p3[b][c] = z[b][c] = f4{0, 0, 0, 0};
            // Chunks of 32 receivers in which one of this wave's two 16-row
            // blocks has a nonzero weight, as wave-uniform bit masks
            // (nch <= 128): a flag load inside the loop would make the MFMAs
            // of a chunk wait for the next chunk's tile, which is issued first.
            uint64_t cm[2] = {0, 0};
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int eb = (ec >> 4) + 2 * we + b, c = 64 * h + lane;
                    const bool on =
                        eb < P.nb && c < nch && (fl[eb * P.nb + 2 * c] | fl[eb * P.nb + 2 * c + 1]) != 0;
                    cm[h] |= __ballot(on);
                }
            // The A fragments of chunk c + 1 are loaded during chunk c, along
            // with its G tile, so the MFMAs of a chunk wait only for LDS.
            auto chunk_on = [&](int rc) {
                const int c = rc / kAdjKC;
                return ((((c < 64) ? cm[0] : cm[1]) >> (c & 63)) & 1) != 0;
            };
            auto load_a = [&](int rc, f4 (&va)[2][2], f4 (&vi)[2][2], f4 (&vw)[2][2]) {
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    // rows beyond mp (when mp is not a multiple of 64) read row
                    // mp - 1: finite values whose products the epilogue drops
                    const int64_t off = (int64_t)min(ec + 32 * we + 16 * b + row, P.mp - 1) * P.mp + rc + 8 * kk;
                    va[b][0] = *reinterpret_cast<const f4 *>(ar + off);
                    va[b][1] = *reinterpret_cast<const f4 *>(ar + off + 4);
                    vi[b][0] = *reinterpret_cast<const f4 *>(ai + off);
                    vi[b][1] = *reinterpret_cast<const f4 *>(ai + off + 4);
                    if (HESS) {
                        vw[b][0] = *reinterpret_cast<const f4 *>(wt + off);
                        vw[b][1] = *reinterpret_cast<const f4 *>(wt + off + 4);
                    }
                }
            };
            auto stage = [&](int rc, float *dst) {
                if (vec)
                    adj_stage_async(gr, gi, P.m, N, rc, x0, dst);
                else
                    adj_stage_regs(gr, gi, P.m, N, rc, x0, dst);
            };
            f4 va[2][2], vi[2][2], vw[2][2];
            stage(0, sB[0]);
            bool on = chunk_on(0);
            if (on) load_a(0, va, vi, vw);
            __builtin_amdgcn_s_waitcnt(0);   // this wave's direct-to-LDS loads have landed
            __syncthreads();
            for (int c = 0; c < nch; ++c) {
                const int rc = c * kAdjKC, buf = c & 1;
                bool on_n = false;
                f4 na[2][2], ni[2][2], nw[2][2];
                if (c + 1 < nch) {
                    stage(rc + kAdjKC, sB[buf ^ 1]);
                    on_n = chunk_on(rc + kAdjKC);
                    if (on_n) load_a(rc + kAdjKC, na, ni, nw);
                }
                if (on) {
                    // a block that is off holds exact zeros in A and W, so it
                    // may be computed along with the other one
                    adj_mma_steps<2, HESS>(va, vi, vw, sB[buf], sB[buf] + kAdjTile, kk, coff, p1, p2, p3, z, 0);
                }
                __builtin_amdgcn_s_waitcnt(0);   // chunk c + 1 has landed in LDS
                __syncthreads();
                on = on_n;
                if (on) {
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            va[b][h] = na[b][h];
                            vi[b][h] = ni[b][h];
                            vw[b][h] = nw[b][h];
                        }
                }
            }
            // fused epilogue: Re sum_e conj(G_e) Y_e and sum_e |G_e|^2 Z_e
#pragma unroll
            for (int b = 0; b < 2; ++b) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = ec + 32 * we + 16 * b + MM<float>::out_row(kk, i);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        const int64_t x = x0 + 32 * wp + 16 * cb + row;
                        const bool ok = (e < P.m) && (x < N);
                        const float ge_r = ok ? gr[(int64_t)e * N + x] : 0.0f;
                        const float ge_i = ok ? gi[(int64_t)e * N + x] : 0.0f;
                        const float yr = p1[b][cb][i] + p2[b][cb][i];
                        const float yi = (p3[b][cb][i] - p1[b][cb][i]) + p2[b][cb][i];
                        gp[cb] += ge_r * yr + ge_i * yi;
                        if (HESS) hp[cb] += (ge_r * ge_r + ge_i * ge_i) * z[b][cb][i];
                    }
                }
            }
        }
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            gacc[cb] += (double)gp[cb] * P.cg[k];
            hacc[cb] += (double)hp[cb] * P.ch[k];
        }
    }
    // lanes of a column (four groups), then the two emitter halves, in a fixed order
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        double g = gacc[cb], h = hacc[cb];
        g += __shfl_xor(g, 16);
        h += __shfl_xor(h, 16);
        g += __shfl_xor(g, 32);
        h += __shfl_xor(h, 32);
        if (kk == 0) {
            sred[we][0][32 * wp + 16 * cb + row] = g;
            sred[we][1][32 * wp + 16 * cb + row] = h;
        }
    }
    __syncthreads();
    if (tid < kAdjNT) {
        const int64_t x = x0 + tid;
        if (x < N) {
            pg[((int64_t)loc.k() * npg + qg) * N + x] = sred[0][0][tid] + sred[1][0][tid];
            if (HESS) ph[((int64_t)loc.k() * npg + qg) * N + x] = sred[0][1][tid] + sred[1][1][tid];
        }
    }
}


// ------------------------------------------------------------------ 16-bit
// |G|^2 of a fragment, rounded to the storage type
template <typename S, typename V>
__device__ __forceinline__ V a16_abs2(V br, V bi) {
    V o;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float a = (float)br[i], b = (float)bi[i];
        o[i] = MM16<S>::from_f(a * a + b * b);
    }
    return o;
}

template <int I>
using Idx = std::integral_constant<int, I>;

// ------------------------------------------------------------------------
// 16-bit backprojection with transposing LDS reads.
//
// Workgroup tile: 128 emitters (a pass; 32 per wave) x 128 pixels, the
// receivers streamed in k-steps of 32.  The G tile of a step (32 receiver
// rows x 128 pixels, both arrays, 16 KB) is copied into LDS by 16-byte direct
// global->LDS loads (one instruction fills four rows), two steps ahead, into
// four buffers.  MFMA B fragments need eight consecutive receivers of one
// pixel per lane; ds_read_b64_tr_b16 delivers four of them from a
// pixel-major tile (within each 16-lane group, lane i receives the i-th
// 16-bit element of the 4 x 8-byte rows its group addressed), so two
// transposing reads give a fragment with no register permutes.  The
// 16-byte chunks of each tile row are XOR-swizzled so that the eight rows
// one half-wave reads together lie on distinct banks; the direct loads
// realise the swizzle by choosing which global chunk each lane fetches.
// A fragments (eight receivers of one emitter) come from L2 as 16-byte
// loads, one step ahead.
//
// Every pass takes the k-steps in the same order, so the passes of a tile
// (adjacent workgroups on one XCD) read each G chunk at about the same time
// and share it in L2.  The epilogue then loads the pass's own emitter rows
// into the freed tile buffers once more and takes G_e from them with the
// same transposing read (four emitters of one pixel per lane).
constexpr int kT16NT = 128;                   // pixels per tile
constexpr int kT16KC = 32;                    // receivers per k-step
constexpr int kT16Row = 2 * kT16NT;           // bytes per tile row
constexpr int kT16Arr = kT16KC * kT16Row;     // bytes of one array of a tile
constexpr int kT16NE = 128;                   // emitters per pass (4 waves x 32)

typedef short t16v4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) t16v4 t16lds_v4;

// chunk position of 16-byte chunk c in tile row r: c XOR 2 g(r), where g
// numbers the rows {0..3, 8..11} (and their shifts by 4 and 16) 0..7
__device__ __forceinline__ int t16_pos(int r, int c) { return c ^ (2 * ((r & 3) | (((r >> 3) & 1) << 2))); }
// byte offset of (tile row r, pixel px) in one array
__device__ __forceinline__ int t16_off(int r, int px) {
    return r * kT16Row + (t16_pos(r, px >> 3) << 4) + ((px & 7) << 1);
}

// Transposing read: lane (group kk, index i) of the wave addresses row
// r0 + (i >> 2), pixels 4 (i & 3) .. + 3 of a 16-pixel column block; it gets
// rows r0 .. r0 + 3 of pixel (i) of the block.
__device__ __forceinline__ t16v4 t16_tr(const unsigned char *p) {
    return __builtin_amdgcn_ds_read_tr16_b64_v4i16((t16lds_v4 *)(p));
}

// The four transposing reads of one column block (rows r and r + 4 of both
// arrays: immediate offsets 0, 4 rows, one array, one array + 4 rows), with
// their wait in the same block.  Written as one asm block so that the
// compiler, which cannot tell these reads from the direct loads filling
// other buffers, adds no wait on those loads here; the k-step's own vmcnt
// wait and barrier order the tile with its reads.
__device__ __forceinline__ void t16_tr4(unsigned addr, t16v4 &a, t16v4 &b, t16v4 &c, t16v4 &d) {
    asm volatile(
        "ds_read_b64_tr_b16 %0, %4\n\t"
        "ds_read_b64_tr_b16 %1, %4 offset:1024\n\t"
        "ds_read_b64_tr_b16 %2, %4 offset:8192\n\t"
        "ds_read_b64_tr_b16 %3, %4 offset:9216\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(a), "=&v"(b), "=&v"(c), "=&v"(d)
        : "v"(addr));
}

template <typename V>
__device__ __forceinline__ V t16_join(t16v4 lo, t16v4 hi) {
    typedef short s8v __attribute__((ext_vector_type(8)));
    const s8v v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(V, v);
}

// Aligned full tiles (N a multiple of 8, m a multiple of 32, 32 N elements
// within 32-bit offsets): wave w issues instructions q = 4 w .. 4 w + 3 of
// the tile's 16 (array q >> 3, rows 4 (q & 7) .. + 3); `goff[j]` is lane l's
// element offset from the step's first row and pixel (`gr`, `gi`: uniform)
// for its j-th instruction, so the loads take a scalar base and a 32-bit
// lane offset.
__device__ __forceinline__ void t16_stage_async(const unsigned short *__restrict__ gr,
                                                const unsigned short *__restrict__ gi, const unsigned (&goff)[4],
                                                unsigned char *sT) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned short *g = (wave >> 1) ? gi : gr;
    unsigned char *d = sT + (wave >> 1) * kT16Arr + (wave & 1) * 4 * 4 * kT16Row;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        __builtin_amdgcn_global_load_lds(g + goff[j], (lds_void_t *)(d + j * 4 * kT16Row), 16, 0, 0);
}

// Ragged or unaligned tiles: through registers, zero beyond m and N; each
// thread writes four 16-byte chunks.
__device__ __forceinline__ void t16_stage_regs(const unsigned short *__restrict__ gr,
                                               const unsigned short *__restrict__ gi, int m, int64_t N, int rc,
                                               int64_t x0, unsigned char *sT) {
#pragma unroll 1
    for (int q = threadIdx.x; q < 2 * kT16KC * 16; q += 256) {
        const int arr = q >> 9, rl = (q >> 4) & 31, pos = q & 15;
        const int c = pos ^ (t16_pos(rl, 0));   // the global chunk stored at `pos`
        const unsigned short *g = arr ? gi : gr;
        const int r = rc + rl;
        unsigned short v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t x = x0 + 8 * c + u;
            v[u] = (r < m && x < N) ? g[(int64_t)r * N + x] : (unsigned short)0;
        }
        unsigned short *d = reinterpret_cast<unsigned short *>(sT + arr * kT16Arr + rl * kT16Row + pos * 16);
#pragma unroll
        for (int u = 0; u < 8; ++u) d[u] = v[u];
    }
}

template <typename S, bool HESS, typename A>
__global__ void __launch_bounds__(256, HESS ? 1 : 2) k_adjoint16_tr(const A args) {
    typename A::Loc loc;
    const AdjItem &it = args.locate(loc);
    const AdjParams &P = it.P;
    const S *__restrict__ Ar = (const S *)it.Ar;
    const S *__restrict__ Ai = (const S *)it.Ai;
    const S *__restrict__ Wt = (const S *)it.Wt;
    const uint8_t *__restrict__ flags = it.flags;
    const float *__restrict__ gscale = it.gscale;
    const float *__restrict__ ascale = it.ascale;
    double *__restrict__ pg = it.pg;
    double *__restrict__ ph = it.ph;
    using V = typename MM16<S>::vec;
    constexpr int EB = 2;   // 16-row emitter blocks per wave
    // four tile buffers as separate LDS objects, addressed by compile-time
    // index inside the k-loop: a direct load into one is then known not to
    // write the one being read
    __shared__ __align__(16) unsigned char sG0[2 * kT16Arr];
    __shared__ __align__(16) unsigned char sG1[2 * kT16Arr];
    __shared__ __align__(16) unsigned char sG2[2 * kT16Arr];
    __shared__ __align__(16) unsigned char sG3[2 * kT16Arr];
    __shared__ float sred[2][4][kT16NT];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kk = lane >> 4;
    const int64_t N = P.N;
    const int k = loc.k();
    const int64_t x0 = (int64_t)loc.tile() * kT16NT;
    const unsigned short *gr = reinterpret_cast<const unsigned short *>((const S *)it.Gr + (int64_t)k * P.m * N);
    const unsigned short *gi = reinterpret_cast<const unsigned short *>((const S *)it.Gi + (int64_t)k * P.m * N);
    const bool vec = ((N & 7) == 0) && (x0 + kT16NT <= N) && (P.m % kT16KC == 0) && N < ((int64_t)1 << 26) &&
                     ((((uintptr_t)gr) | ((uintptr_t)gi)) & 15) == 0;   // workgroup-uniform
    const S *ar = Ar + (int64_t)k * P.mp * P.mp;
    const S *ai = Ai + (int64_t)k * P.mp * P.mp;
    const S *wt = Wt + (int64_t)k * P.mp * P.mp;
    const uint8_t *fl = flags + (int64_t)k * P.nb * P.nb;
    const int nch = P.mp / kT16KC;
    // lane's element offsets of its four direct-load chunks within a step
    unsigned goff[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int rl = 4 * (4 * (wave & 1) + j) + (lane >> 4);
        goff[j] = (unsigned)(rl * N) + 8u * (unsigned)((lane & 15) ^ (t16_pos(rl, 0)));
    }
    // transposing-read offsets: rows 8 kk + 4 h + (row >> 2), pixels
    // 16 cb + 4 (row & 3) (h = 0, 1; cb = 0 .. 7)
    int toff[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) toff[h][cb] = t16_off(8 * kk + 4 * h + (row >> 2), 16 * cb + 4 * (row & 3));
    float gp[8], hp[8];
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) gp[cb] = hp[cb] = 0.0f;
    auto buf = [&](auto itag) -> unsigned char * {
        constexpr int I = decltype(itag)::value & 3;
        return I == 0 ? sG0 : (I == 1 ? sG1 : (I == 2 ? sG2 : sG3));
    };

    const int npass = (P.mp + kT16NE - 1) / kT16NE, npg = it.npg, qg = loc.group();
    const int pass0 = qg * npass / npg, pass1 = (qg + 1) * npass / npg;
    for (int ec = pass0 * kT16NE; ec < pass1 * kT16NE; ec += kT16NE) {
        const int e0 = ec + 32 * wave;
        // every pass takes the receiver chunks in the same order, so that the
        // passes of a tile (adjacent workgroups on one XCD) read each G chunk
        // at about the same time and share it in L2
        // (opaque to the compiler, which would otherwise keep a strength-
        // reduced address per unrolled step live in registers)
        auto chunk = [&](int s) {
            asm volatile("" : "+s"(s));
            return s;
        };
        f4 yr[EB][8], yn[EB][8], z[EB][8];
#pragma unroll
        for (int b = 0; b < EB; ++b)
#pragma unroll
            for (int cb = 0; cb < 8; ++cb) yr[b][cb] = yn[b][cb] = z[b][cb] = f4{0, 0, 0, 0};
        unsigned aoff[EB];
#pragma unroll
        for (int b = 0; b < EB; ++b) aoff[b] = (unsigned)(min(e0 + 16 * b + row, P.mp - 1) * P.mp + 8 * kk);
        auto load_a = [&](int c, V (&va)[EB], V (&vi)[EB], V (&vw)[EB]) {
            const int co = c * kT16KC;   // uniform
#pragma unroll
            for (int b = 0; b < EB; ++b) {
                va[b] = *reinterpret_cast<const V *>(ar + co + aoff[b]);
                vi[b] = *reinterpret_cast<const V *>(ai + co + aoff[b]);
                if (HESS) vw[b] = *reinterpret_cast<const V *>(wt + co + aoff[b]);
            }
        };
        // chunks in which a 16-row block of this wave has a nonzero weight
        uint64_t cm[2] = {0, 0};
#pragma unroll
        for (int b = 0; b < EB; ++b)
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int eb = (e0 >> 4) + b, c = 64 * hh + lane;
                const bool on =
                    eb < P.nb && c < nch && (fl[eb * P.nb + 2 * c] | fl[eb * P.nb + 2 * c + 1]) != 0;
                cm[hh] |= __ballot(on);
            }
        auto stage = [&](int c, unsigned char *dst, auto vtag) {
            if (decltype(vtag)::value)
                t16_stage_async(gr + ((int64_t)c * kT16KC * N + x0), gi + ((int64_t)c * kT16KC * N + x0), goff, dst);
            else
                t16_stage_regs(gr, gi, P.m, N, c * kT16KC, x0, dst);
        };
        // One k-step s (chunk c = chunk(s)) on the tile in buffer s mod 4:
        // wait for its tile and A(c), issue A(next) and the tile of step
        // s + 2, then the MFMAs.  Per step a wave issues A(s + 1) (2 EB or
        // 3 EB loads) and then the tile of s + 2 (4 direct loads), so at the
        // wait only the tile of s + 1 may still be in flight.  `mode` says
        // what the step issues when that is known at compile time (3: A and
        // a tile, 2: A only, 1: nothing; 0: decided from s at run time), so
        // that the compiler's own load-counter waits stay exact.
        auto kstep = [&](int s, auto itag, V (&va)[EB], V (&vi)[EB], V (&vw)[EB], V (&na)[EB], V (&ni)[EB],
                         V (&nw)[EB], auto vtag, auto mode) {
            constexpr int I = decltype(itag)::value;
            constexpr int M = decltype(mode)::value;
            const bool has_a = M == 3 || M == 2 || (M == 0 && s + 1 < nch);
            const bool has_t = M == 3 || (M == 0 && s + 2 < nch);
            if (has_a)
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(4));   // tile s + 1
            else
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            lds_barrier();
            const int c = chunk(s);
            if (has_a) load_a(chunk(s + 1), na, ni, nw);
            __builtin_amdgcn_sched_barrier(0);
            if (has_t) stage(chunk(s + 2), buf(Idx<I + 2>()), vtag);
            __builtin_amdgcn_sched_barrier(0);
            if (!(((c < 64 ? cm[0] : cm[1]) >> (c & 63)) & 1)) return;
            const unsigned char *sb = buf(Idx<I>());
            V nva[EB];
#pragma unroll
            for (int b = 0; b < EB; ++b) nva[b] = neg(vi[b]);
            const unsigned sba = (unsigned)(uintptr_t)(const __attribute__((address_space(3))) unsigned char *)sb;
#pragma unroll
            for (int cb = 0; cb < 8; ++cb) {
                t16v4 r0, r1, i0, i1;
                t16_tr4(sba + (unsigned)toff[0][cb], r0, r1, i0, i1);
                const V br = t16_join<V>(r0, r1);
                const V bi = t16_join<V>(i0, i1);
                V b2;
                if (HESS) b2 = a16_abs2<S, V>(br, bi);
#pragma unroll
                for (int b = 0; b < EB; ++b) {
                    yr[b][cb] = MM16<S>::mma(va[b], br, yr[b][cb]);
                    yr[b][cb] = MM16<S>::mma(vi[b], bi, yr[b][cb]);
                    yn[b][cb] = MM16<S>::mma(va[b], bi, yn[b][cb]);
                    yn[b][cb] = MM16<S>::mma(nva[b], br, yn[b][cb]);
                    if (HESS) z[b][cb] = MM16<S>::mma(vw[b], b2, z[b][cb]);
                }
            }
        };
        // the k-loop, specialised on the staging path and unrolled by four
        // (buffer index period 4, A registers period 2); the steady state
        // has no conditional steps, the last two to five follow.  (Making
        // those compile-time as well spills the accumulators.)
        auto kloop = [&](auto vtag) {
            using M3 = std::integral_constant<int, 3>;
            using M2 = std::integral_constant<int, 2>;
            using M1 = std::integral_constant<int, 1>;
            using M0 = std::integral_constant<int, 0>;
            V va[EB], vi[EB], vw[EB], na[EB], ni[EB], nw[EB];
            lds_barrier();   // the previous pass is done with the tile buffers
            stage(chunk(0), sG0, vtag);
            load_a(chunk(0), va, vi, vw);
            // unconditional (a one-chunk pass stages its chunk twice), so that
            // the loop is always entered with the same loads in flight and
            // the compiler's load-counter waits at its head stay exact
            stage(chunk(min(1, nch - 1)), sG1, vtag);
            int s = 0;
            for (; s + 6 <= nch; s += 4) {
                kstep(s, Idx<0>(), va, vi, vw, na, ni, nw, vtag, M3());
                kstep(s + 1, Idx<1>(), na, ni, nw, va, vi, vw, vtag, M3());
                kstep(s + 2, Idx<2>(), va, vi, vw, na, ni, nw, vtag, M3());
                kstep(s + 3, Idx<3>(), na, ni, nw, va, vi, vw, vtag, M3());
            }
            if (s < nch) kstep(s, Idx<0>(), va, vi, vw, na, ni, nw, vtag, M0());
            if (s + 1 < nch) kstep(s + 1, Idx<1>(), na, ni, nw, va, vi, vw, vtag, M0());
            if (s + 2 < nch) kstep(s + 2, Idx<2>(), va, vi, vw, na, ni, nw, vtag, M0());
            if (s + 3 < nch) kstep(s + 3, Idx<3>(), na, ni, nw, va, vi, vw, vtag, M0());
            if (s + 4 < nch) kstep(s + 4, Idx<0>(), va, vi, vw, na, ni, nw, vtag, M0());
            // keep the epilogue's work out of the last k-steps' schedule
            __builtin_amdgcn_sched_barrier(0);
        };
        if (vec)
            kloop(std::true_type());
        else
            kloop(std::false_type());
        // fused epilogue: Re sum_e conj(G_e) Y_e and sum_e |G_e|^2 Z_e.  The
        // tile buffers are free once every wave is done with the k-loop:
        // wave w copies the chunk of its 32 emitter rows (both arrays) into
        // buffer w again, and a transposing read at rows 16 b + 4 kk gives
        // lane (kk, row) emitters 16 b + 4 kk + i (i = 0..3) of pixel
        // 16 cb + row, the layout of the accumulators (zero beyond m and N).
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        lds_barrier();
        unsigned char *se = wave == 0 ? sG0 : (wave == 1 ? sG1 : (wave == 2 ? sG2 : sG3));
        if (vec) {
            if (e0 < P.mp) {
                const unsigned short *g0 = gr + ((int64_t)e0 * N + x0), *g1 = gi + ((int64_t)e0 * N + x0);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int rl = 4 * (q & 7) + (lane >> 4);
                    const unsigned go = (unsigned)(rl * N) + 8u * (unsigned)((lane & 15) ^ t16_pos(rl, 0));
                    __builtin_amdgcn_global_load_lds((q >> 3) ? g1 + go : g0 + go,
                                                     (lds_void_t *)(se + (q >> 3) * kT16Arr + 4 * (q & 7) * kT16Row),
                                                     16, 0, 0);
                }
            }
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        } else {
            t16_stage_regs(gr, gi, P.m, N, ec, x0, sG0);
            t16_stage_regs(gr, gi, P.m, N, ec + kT16KC, x0, sG1);
            t16_stage_regs(gr, gi, P.m, N, ec + 2 * kT16KC, x0, sG2);
            t16_stage_regs(gr, gi, P.m, N, ec + 3 * kT16KC, x0, sG3);
        }
        lds_barrier();
        if (e0 < P.mp) {
#pragma unroll
            for (int b = 0; b < EB; ++b) {
#pragma unroll
                for (int cb = 0; cb < 8; ++cb) {
                    const int off = t16_off(16 * b + 4 * kk + (row >> 2), 16 * cb + 4 * (row & 3));
                    const t16v4 vr = t16_tr(se + off), vi = t16_tr(se + kT16Arr + off);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const bool ok = e0 + 16 * b + 4 * kk + i < P.m;
                        const float ger = ok ? MM16<S>::bits_to_f((unsigned short)vr[i]) : 0.0f;
                        const float gei = ok ? MM16<S>::bits_to_f((unsigned short)vi[i]) : 0.0f;
                        gp[cb] += ger * yr[b][cb][i] - gei * yn[b][cb][i];
                        if (HESS) hp[cb] += (ger * ger + gei * gei) * z[b][cb][i];
                    }
                }
            }
        }
    }
    // the four lane groups of a column, then the waves, in a fixed order
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) {
        float g = gp[cb], h = hp[cb];
        g += __shfl_xor(g, 16);
        h += __shfl_xor(h, 16);
        g += __shfl_xor(g, 32);
        h += __shfl_xor(h, 32);
        if (kk == 0) {
            sred[0][wave][16 * cb + row] = g;
            sred[1][wave][16 * cb + row] = h;
        }
    }
    __syncthreads();
    if (tid < kT16NT) {
        const int64_t x = x0 + tid;
        if (x < N) {
            const double gs = (double)gscale[k], as = ascale[k] > 0.0f ? (double)ascale[k] : 1.0;
            const double g2 = gs * gs;
            double g = 0.0, h = 0.0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                g += (double)sred[0][w][tid];
                h += (double)sred[1][w][tid];
            }
            const int npgl = it.npg;
            pg[((int64_t)k * npgl + qg) * N + x] = g * (P.cg[k] * g2 * as);
            if (HESS) ph[((int64_t)k * npgl + qg) * N + x] = h * (P.ch[k] * g2 * g2);
        }
    }
}


// grad += sum_k sum_q pg[k][q], hd += sum_k sum_q ph[k][q] in frequency
// order, then emitter-pass group order.
__global__ void k_adj_sum(int64_t N, int nf, int npg, const double *__restrict__ pg, const double *__restrict__ ph,
                          double *__restrict__ grad, double *__restrict__ hd) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    double g = 0.0, h = 0.0;
    for (int k = 0; k < nf * npg; ++k) {
        g += pg[(int64_t)k * N + x];
        if (hd) h += ph[(int64_t)k * N + x];
    }
    grad[x] += g;
    if (hd) hd[x] += h;
}

}  // namespace

// ---------------------------------------------------------------- host side
// rows/columns of the adjoint operands are padded to a multiple of 32
static int pad_m(int m) { return (m + 31) / 32 * 32; }

static AdjParams adj_params(const rb_geometry *g, const double *freqs, int nf) {
    AdjParams P;
    P.m = g->m;
    P.mp = pad_m(g->m);
    P.nb = P.mp / 16;
    P.N = (int64_t)g->nx * g->ny;
    P.nf = nf;
    const double dA = g->h * g->h;
    for (int k = 0; k < nf; ++k) {
        const double om = 2.0 * M_PI * freqs[k];
        const double c = om * om * dA;
        P.cg[k] = c;
        P.ch[k] = c * c;
    }
    return P;
}

struct AdjWs {
    void *Ar, *Ai, *Wt;
    uint8_t *flags;
    float *ascale;
    double *pg, *ph;  // per-frequency partials of the f32 backprojection
};

// Workgroups that split the emitter passes of one pixel tile: every pass
// (64 emitters in the FP32 kernel, 128 in the 16-bit one) goes to a
// workgroup of its own once there are four or more, the passes of a tile
// adjacent in logical order and on one XCD (AdjOneSplit), so that the
// tile's G rows come from HBM once and from L2 for the other passes (FP32,
// 1024 elements / 1100^2: 221.6 -> 209.6 ms per 4-frequency launch; 16-bit:
// 51.9 -> 47.6 ms).  Ordering the split workgroups pass-major instead (all
// workgroups in flight on one pass, sharing its W.D rows) was slower: 224.7
// and 60.0 ms; so was nothing in between: dealing a tile's groups into 2
// or 4 subsets on their own XCDs (each L2 then holds a half or a quarter of
// W.D) left the launches at 211.8 / 212.3 ms (FP32, from 211.5) and 33.2 /
// 33.4 ms (16-bit, from 33.5).  One workgroup per tile otherwise.
static int adj_groups(const rb_geometry *g, rb_dtype dt) {
    if (dt == RB_F32) {
        const int npass = (pad_m(g->m) + 63) / 64;   // 64 emitters per pass of k_adjoint_f32
        return npass >= 4 ? npass : 1;
    }
    if (dt != RB_BF16 && dt != RB_F16) return 1;
    const int ne = kT16NE;   // emitters per pass of k_adjoint16_tr
    const int npass = (pad_m(g->m) + ne - 1) / ne;
    return npass >= 4 ? npass : 1;
}

static AdjWs carve_adj(Carver &c, const rb_geometry *g, int nf, rb_dtype dt) {
    const int mp = pad_m(g->m);
    const size_t npg = (size_t)adj_groups(g, dt);
    const size_t per = (size_t)nf * mp * mp;
    const size_t es = dt == RB_F64 ? 8 : (dt == RB_F32 ? 4 : 2);
    AdjWs w;
    w.Ar = c.take<char>(per * es);
    w.Ai = c.take<char>(per * es);
    w.Wt = c.take<char>(per * es);
    w.flags = c.take<uint8_t>((size_t)nf * (mp / 16) * (mp / 16));
    w.ascale = c.take<float>(RB_MAX_NF);
    w.pg = c.take<double>((size_t)nf * npg * g->nx * g->ny);
    w.ph = c.take<double>((size_t)nf * npg * g->nx * g->ny);
    return w;
}

size_t adjoint_workspace_bytes(const rb_geometry *g, int nf, rb_dtype dt) {
    Carver c(nullptr, 0);
    carve_adj(c, g, nf, dt);
    return c.used + 256;
}

rb_status adjoint_prepare(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                          rb_dtype dt, const double *freqs, int nf, const double *d_res, const double *w_data,
                          double *grad, double *hdiag, void *ws, size_t ws_bytes, hipStream_t st, AdjTask *task) {
    if (ws_bytes < adjoint_workspace_bytes(g, nf, dt)) {
        set_error("adjoint workspace too small: need %zu bytes", adjoint_workspace_bytes(g, nf, dt));
        return RB_ENOMEM;
    }
    Carver c(ws, ws_bytes);
    AdjWs w = carve_adj(c, g, nf, dt);
    AdjParams P = adj_params(g, freqs, nf);
    const int64_t tot = (int64_t)nf * P.mp * P.mp;
    const unsigned bp = (unsigned)std::min<int64_t>(blocks_for(tot, 256), 8192);
    const bool scaled = (dt == RB_BF16 || dt == RB_F16);
    if (scaled) RB_TRY(fill_f32(w.ascale, 0.0f, nf, st));
    k_adj_blocks<<<dim3(P.nb * P.nb, nf), 256, 0, st>>>(g->m, P.nb, d_res, w_data, w.flags,
                                                        scaled ? reinterpret_cast<unsigned *>(w.ascale) : nullptr);
    RB_LAUNCHED();
    switch (dt) {
        case RB_F64:
            k_adj_prep<double, false><<<bp, 256, 0, st>>>(g->m, P.mp, nf, d_res, w_data, nullptr, (double *)w.Ar,
                                                          (double *)w.Ai, (double *)w.Wt);
            break;
        case RB_F32:
            k_adj_prep<float, false, true><<<bp, 256, 0, st>>>(g->m, P.mp, nf, d_res, w_data, nullptr,
                                                               (float *)w.Ar, (float *)w.Ai, (float *)w.Wt);
            break;
        case RB_BF16:
            k_adj_prep<__hip_bfloat16, true><<<bp, 256, 0, st>>>(g->m, P.mp, nf, d_res, w_data, w.ascale,
                                                                 (__hip_bfloat16 *)w.Ar, (__hip_bfloat16 *)w.Ai,
                                                                 (__hip_bfloat16 *)w.Wt);
            break;
        case RB_F16:
            k_adj_prep<__half, true><<<bp, 256, 0, st>>>(g->m, P.mp, nf, d_res, w_data, w.ascale, (__half *)w.Ar,
                                                         (__half *)w.Ai, (__half *)w.Wt);
            break;
    }
    RB_LAUNCHED();
    AdjItem &it = task->item;
    it.P = P;
    it.Gr = G_re;
    it.Gi = G_im;
    it.Ar = w.Ar;
    it.Ai = w.Ai;
    it.Wt = w.Wt;
    it.flags = w.flags;
    it.gscale = gscale;
    it.ascale = w.ascale;
    it.pg = w.pg;
    it.ph = w.ph;
    it.ntiles = (int)blocks_for(P.N, dt == RB_F32 ? kAdjNT : kT16NT);
    it.begin = 0;
    it.npg = adj_groups(g, dt);
    task->dt = dt;
    task->grad = grad;
    task->hdiag = hdiag;
    return RB_OK;
}

rb_status adjoint_run(const AdjTask &task, hipStream_t st) {
    const AdjItem &it = task.item;
    const AdjParams &P = it.P;
    const int nf = P.nf;
    double *grad = task.grad, *hdiag = task.hdiag;
    switch (task.dt) {
        case RB_F64: {
            const unsigned nb = blocks_for(P.N, 64 * 2);
            k_adjoint<double, 2, 2><<<nb, 256, 0, st>>>(P, (const double *)it.Gr, (const double *)it.Gi,
                                                        (const double *)it.Ar, (const double *)it.Ai,
                                                        (const double *)it.Wt, it.flags, grad, hdiag);
            break;
        }
        case RB_F32: {
            if (it.npg == 1) {
                dim3 ga(blocks_for(P.N, kAdjNT), nf);
                const AdjOne one{it};
                if (hdiag)
                    k_adjoint_f32<true><<<ga, 256, 0, st>>>(one);
                else
                    k_adjoint_f32<false><<<ga, 256, 0, st>>>(one);
            } else {
                dim3 ga((unsigned)it.ntiles * it.npg, nf);
                const AdjOneSplit one{it};
                if (hdiag)
                    k_adjoint_f32<true><<<ga, 256, 0, st>>>(one);
                else
                    k_adjoint_f32<false><<<ga, 256, 0, st>>>(one);
            }
            RB_LAUNCHED();
            k_adj_sum<<<blocks_for(P.N, 256), 256, 0, st>>>(P.N, nf, it.npg, it.pg, it.ph, grad, hdiag);
            break;
        }
        case RB_BF16:
        case RB_F16: {
            dim3 ga((unsigned)it.ntiles * it.npg, nf);
            const AdjOneSplit one{it};
            auto go = [&](auto tag) {
                using S = decltype(tag);
                if (hdiag)
                    k_adjoint16_tr<S, true><<<ga, 256, 0, st>>>(one);
                else
                    k_adjoint16_tr<S, false><<<ga, 256, 0, st>>>(one);
            };
            if (task.dt == RB_BF16)
                go(__hip_bfloat16());
            else
                go(__half());
            RB_LAUNCHED();
            k_adj_sum<<<blocks_for(P.N, 256), 256, 0, st>>>(P.N, nf, it.npg, it.pg, it.ph, grad, hdiag);
            break;
        }
    }
    RB_LAUNCHED();
    return RB_OK;
}

rb_status adjoint_run_grouped(AdjTask *const *tasks, int n, hipStream_t st) {
    // contraction type and variant of a task: f32 / bf16 / f16, with or
    // without the Hessian diagonal; f64 runs alone
    auto kind = [](const AdjTask &t) { return 2 * (int)t.dt + (t.hdiag ? 1 : 0); };
    bool done[256] = {};
    RB_CHECK_ARG(n >= 0 && n <= 256, "grouped backprojection: %d problems (at most 256)", n);
    for (int i = 0; i < n; ++i) {
        if (done[i]) continue;
        if (tasks[i]->dt == RB_F64) {
            RB_TRY(adjoint_run(*tasks[i], st));
            done[i] = true;
            continue;
        }
        // up to kAdjGroupMax not-yet-run tasks of this kind, in order
        AdjGroupArg arg;
        AdjGroup &G = arg.G;
        G.n = 0;
        int idx[kAdjGroupMax];
        int64_t blocks = 0;
        for (int j = i; j < n && G.n < kAdjGroupMax; ++j) {
            if (done[j] || kind(*tasks[j]) != kind(*tasks[i])) continue;
            AdjItem it = tasks[j]->item;
            it.begin = (int)blocks;
            blocks += (int64_t)it.ntiles * it.npg * it.P.nf;
            G.item[G.n] = it;
            idx[G.n++] = j;
            done[j] = true;
        }
        RB_CHECK_ARG(blocks < (int64_t)1 << 31, "grouped backprojection: too many workgroups");
        const bool hess = tasks[i]->hdiag != nullptr;
        switch (tasks[i]->dt) {
            case RB_F32:
                if (hess)
                    k_adjoint_f32<true><<<(unsigned)blocks, 256, 0, st>>>(arg);
                else
                    k_adjoint_f32<false><<<(unsigned)blocks, 256, 0, st>>>(arg);
                break;
            case RB_BF16:
                if (hess)
                    k_adjoint16_tr<__hip_bfloat16, true><<<(unsigned)blocks, 256, 0, st>>>(arg);
                else
                    k_adjoint16_tr<__hip_bfloat16, false><<<(unsigned)blocks, 256, 0, st>>>(arg);
                break;
            case RB_F16:
                if (hess)
                    k_adjoint16_tr<__half, true><<<(unsigned)blocks, 256, 0, st>>>(arg);
                else
                    k_adjoint16_tr<__half, false><<<(unsigned)blocks, 256, 0, st>>>(arg);
                break;
            default:
                break;
        }
        RB_LAUNCHED();
        for (int q = 0; q < G.n; ++q) {
            const AdjTask &t = *tasks[idx[q]];
            k_adj_sum<<<blocks_for(t.item.P.N, 256), 256, 0, st>>>(t.item.P.N, t.item.P.nf, t.item.npg, t.item.pg,
                                                                   t.item.ph, t.grad, t.hdiag);
            RB_LAUNCHED();
        }
    }
    return RB_OK;
}

rb_status adjoint_impl(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                       rb_dtype dt, const double *freqs, int nf, const double *d_res, const double *w_data,
                       double *grad, double *hdiag, void *ws, size_t ws_bytes, hipStream_t st) {
    AdjTask task;
    RB_TRY(adjoint_prepare(g, G_re, G_im, gscale, dt, freqs, nf, d_res, w_data, grad, hdiag, ws, ws_bytes, st,
                           &task));
    return adjoint_run(task, st);
}

// ---------------------------------------------------------------- no-allocation variant
// Scratch of rb_born_adjoint_weighted_noalloc: the same workspace the
// ordinary entry point carves from its caller's buffer, held in one device
// array per GPU (allocated when the library is loaded on that GPU and kept
// until the process ends).  Host code never passes `scratch` itself to a
// kernel: its name there is a host-side stand-in; the device address comes
// from hipGetSymbolAddress, looked up once per device.
static __device__ __align__(256) unsigned char scratch[RB_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device.
static rb_status scratch_address(void **out) {
    int dev = 0;
    RB_HIP(hipGetDevice(&dev));
    RB_CHECK_ARG(dev >= 0 && dev < kMaxDevices, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        RB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RB_OK;
}

}  // namespace rb

extern "C" {

size_t rb_adjoint_workspace_bytes(const rb_geometry *g, int32_t nf, rb_dtype dtype) {
    if (rb::check_geometry(g) != RB_OK || nf < 1 || nf > RB_MAX_NF) return 0;
    return rb::adjoint_workspace_bytes(g, nf, dtype);
}

rb_status rb_born_adjoint_weighted(const rb_geometry *g, const void *G_re, const void *G_im, const float *scale,
                                   rb_dtype dtype, const double *freqs_hz, int32_t nf, const double *d_res,
                                   const double *w_data, double *grad, double *hdiag, void *ws, size_t ws_bytes,
                                   void *stream) {
    rb::clear_error();
    RB_TRY(rb::check_contraction(g, G_re, G_im, scale, dtype, freqs_hz, nf));
    RB_CHECK_ARG(d_res && w_data && grad, "d_res/w_data/grad are NULL");
    RB_CHECK_ARG(ws, "workspace is NULL");
    return rb::adjoint_impl(g, G_re, G_im, scale, dtype, freqs_hz, nf, d_res, w_data, grad, hdiag, ws, ws_bytes,
                            rb::as_stream(stream));
}

rb_status rb_born_adjoint_weighted_noalloc(const rb_geometry *g, const void *G_re, const void *G_im,
                                           const float *scale, rb_dtype dtype, const double *freqs_hz,
                                           int32_t nf, const double *d_res, const double *w_data, double *grad,
                                           double *hdiag, void *stream) {
    rb::clear_error();
    RB_TRY(rb::check_contraction(g, G_re, G_im, scale, dtype, freqs_hz, nf));
    RB_CHECK_ARG(d_res && w_data && grad, "d_res/w_data/grad are NULL");
    const size_t need = rb::adjoint_workspace_bytes(g, nf, dtype);
    if (need > (size_t)RB_NOALLOC_SCRATCH_BYTES) {
        rb::set_error("rb_born_adjoint_weighted_noalloc: this problem needs %zu bytes of scratch, the fixed "
                      "scratch holds %zu (use rb_born_adjoint_weighted with a workspace)",
                      need, (size_t)RB_NOALLOC_SCRATCH_BYTES);
        return RB_ENOMEM;
    }
    void *ws = nullptr;
    RB_TRY(rb::scratch_address(&ws));
    return rb::adjoint_impl(g, G_re, G_im, scale, dtype, freqs_hz, nf, d_res, w_data, grad, hdiag, ws,
                            (size_t)RB_NOALLOC_SCRATCH_BYTES, rb::as_stream(stream));
}

}  // extern "C"
