// Born forward operator and weighted adjoint (backprojection) with the
// diagonal of the Gauss-Newton Hessian (paper, Inverse Problem section,
// Eqs. 8-10; linearisation of Eq. 1 in q = 1/c^2 with Green's functions from
// Eqs. 4-5).
//
//   forward:  d_er = omega^2 h^2 sum_x G_e(x) G_r(x) delta(x)
//   adjoint:  grad(x) = omega^2 h^2 Re sum_e conj(G_e(x)) Y_e(x),
//             Y_e(x)  = sum_r A_er conj(G_r(x)),      A = W . D
//   Hessian:  hd(x)   = omega^4 h^4 sum_e |G_e(x)|^2 Z_e(x),
//             Z_e(x)  = sum_r W_er |G_r(x)|^2
//
// Both are dense contractions over emitter x receiver pairs, so they run on
// the matrix cores.  Complex products are expanded into real MFMAs:
//   Yr  = Ar.Gr + Ai.Gi,   -Yi = Ar.Gi + (-Ai).Gr,   Z = W.|G|^2
// and the reduction over e against G_e(x) is fused into the epilogue, so Y
// and Z never leave registers.  A k-permutation (lane group kk supplies
// k = 4 kk + s at MFMA step s) lets each lane fetch its A fragment with one
// vector load.  Blocks of A whose weights are all zero (the receiver
// selection removes a band around the diagonal) are skipped per 16x16 block.
// The forward operator is a split-K GEMM over pixels whose symmetric output
// is computed on upper-triangular tiles only and reduced in a fixed order.
#include <algorithm>
#include <cmath>

#include "born.h"
#include "common.h"

namespace rb {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

template <typename T>
struct MM;
// Both 16x16x4 forms read A[i][k] from lane i + 16k and B[k][j] from lane
// j + 16k.  Output element `i` of lane group kk (lanes 16kk..16kk+15, column
// = lane % 16) holds row 4kk + i for f32 but row kk + 4i for f64 (measured).
template <>
struct MM<float> {
    using acc = f4;
    __device__ __forceinline__ static acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int out_row(int kk, int i) { return 4 * kk + i; }
};
template <>
struct MM<double> {
    using acc = d4;
    __device__ __forceinline__ static acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int out_row(int kk, int i) { return kk + 4 * i; }
};

// 16-bit storage types and their MFMA (16x16x32, 8 k-values per lane).
template <typename S>
struct MM16;
template <>
struct MM16<__hip_bfloat16> {
    using vec = bf8;
    __device__ __forceinline__ static f4 mma(vec a, vec b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static float to_f(__hip_bfloat16 v) { return __bfloat162float(v); }
    __device__ __forceinline__ static __bf16 from_f(float v) {
        __hip_bfloat16 b = __float2bfloat16(v);
        return *reinterpret_cast<__bf16 *>(&b);
    }
};
template <>
struct MM16<__half> {
    using vec = h8;
    __device__ __forceinline__ static f4 mma(vec a, vec b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static float to_f(__half v) { return __half2float(v); }
    __device__ __forceinline__ static _Float16 from_f(float v) { return (_Float16)v; }
};

typedef short s8 __attribute__((ext_vector_type(8)));
// sign flip of eight 16-bit floats (bf16 and fp16 keep the sign in bit 15)
template <typename V>
__device__ __forceinline__ V neg(V v) {
    s8 b = __builtin_bit_cast(s8, v);
    b ^= (short)0x8000;
    return __builtin_bit_cast(V, b);
}

template <typename T>
__device__ __forceinline__ T ld(const T *p, bool ok) {
    return ok ? p[0] : T(0);
}

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

// 16-bit variant: MFMA 16x16x32 with FP32 accumulation.  Lane group kk
// supplies k = 8 kk + i (i = 0..7); operands are stored pre-scaled.
template <typename S, int RB, int CB>
__global__ void __launch_bounds__(256) k_adjoint16(AdjParams P, const S *__restrict__ Gr, const S *__restrict__ Gi,
                                                   const S *__restrict__ Ar, const S *__restrict__ Ai,
                                                   const S *__restrict__ Wt, const uint8_t *__restrict__ flags,
                                                   const float *__restrict__ gscale,
                                                   const float *__restrict__ ascale, double *__restrict__ grad,
                                                   double *__restrict__ hd) {
    using V = typename MM16<S>::vec;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kk = lane >> 4;
    const int64_t N = P.N;
    const int64_t xw = (int64_t)blockIdx.x * (64 * CB) + (int64_t)wave * 16 * CB;
    double gacc[CB], hacc[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) gacc[c] = hacc[c] = 0.0;

    for (int k = 0; k < P.nf; ++k) {
        const S *gr = Gr + (int64_t)k * P.m * N;
        const S *gi = Gi + (int64_t)k * P.m * N;
        const S *ar = Ar + (int64_t)k * P.mp * P.mp;
        const S *ai = Ai + (int64_t)k * P.mp * P.mp;
        const S *wt = Wt + (int64_t)k * P.mp * P.mp;
        const uint8_t *fl = flags + (int64_t)k * P.nb * P.nb;
        float gp[CB], hp[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) gp[c] = hp[c] = 0.0f;
        for (int ec = 0; ec < P.mp; ec += 16 * RB) {
            f4 yr[RB][CB], yn[RB][CB], z[RB][CB];
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int c = 0; c < CB; ++c) yr[b][c] = yn[b][c] = z[b][c] = f4{0, 0, 0, 0};
            for (int rc = 0; rc < P.mp; rc += 32) {
                bool on[RB];
                bool any = false;
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    const int eb = ec / 16 + b;
                    on[b] = (eb < P.nb) && (fl[eb * P.nb + rc / 16] || fl[eb * P.nb + rc / 16 + 1]);
                    any |= on[b];
                }
                if (!any) continue;
                V br[CB], bi[CB], b2[CB];
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    const int64_t x = xw + 16 * c + row;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int r = rc + 8 * kk + i;
                        const bool ok = (r < P.m) && (x < N);
                        const float fr = ok ? MM16<S>::to_f(gr[(int64_t)r * N + x]) : 0.0f;
                        const float fi = ok ? MM16<S>::to_f(gi[(int64_t)r * N + x]) : 0.0f;
                        br[c][i] = MM16<S>::from_f(fr);
                        bi[c][i] = MM16<S>::from_f(fi);
                        b2[c][i] = MM16<S>::from_f(fr * fr + fi * fi);
                    }
                }
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    if (!on[b]) continue;
                    const int64_t off = (int64_t)(ec + 16 * b + row) * P.mp + rc + 8 * kk;
                    const V va = *reinterpret_cast<const V *>(ar + off);
                    const V vi = *reinterpret_cast<const V *>(ai + off);
                    const V vw = *reinterpret_cast<const V *>(wt + off);
                    const V vn = neg(vi);
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        yr[b][c] = MM16<S>::mma(va, br[c], yr[b][c]);
                        yr[b][c] = MM16<S>::mma(vi, bi[c], yr[b][c]);
                        yn[b][c] = MM16<S>::mma(va, bi[c], yn[b][c]);
                        yn[b][c] = MM16<S>::mma(vn, br[c], yn[b][c]);
                        z[b][c] = MM16<S>::mma(vw, b2[c], z[b][c]);
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < RB; ++b) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = ec + 16 * b + 4 * kk + i;
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        const int64_t x = xw + 16 * c + row;
                        const bool ok = (e < P.m) && (x < N);
                        const float ge_r = ok ? MM16<S>::to_f(gr[(int64_t)e * N + x]) : 0.0f;
                        const float ge_i = ok ? MM16<S>::to_f(gi[(int64_t)e * N + x]) : 0.0f;
                        gp[c] += ge_r * yr[b][c][i] - ge_i * yn[b][c][i];
                        hp[c] += (ge_r * ge_r + ge_i * ge_i) * z[b][c][i];
                    }
                }
            }
        }
        const double gs = (double)gscale[k], as = (double)ascale[k];
        const double g2 = gs * gs;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            gacc[c] += (double)gp[c] * (P.cg[k] * g2 * as);
            hacc[c] += (double)hp[c] * (P.ch[k] * g2 * g2);
        }
    }
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
// = max |W D| (W is 0/1-valued in the inversion, stored unscaled).
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

__global__ void k_adj_absmax(int m, const double *__restrict__ d, const double *__restrict__ w,
                             float *__restrict__ ascale) {
    // one block per frequency
    __shared__ double sh[256];
    const int k = blockIdx.x;
    const int64_t mm = (int64_t)m * m;
    double best = 0.0;
    for (int64_t i = threadIdx.x; i < mm; i += 256) {
        const int64_t q = (int64_t)k * mm + i;
        const double wv = w[q];
        const double re = wv * d[2 * q], im = wv * d[2 * q + 1];
        best = fmax(best, fmax(fabs(re), fabs(im)));
    }
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) ascale[k] = sh[0] > 0.0 ? (float)sh[0] : 1.0f;
}

// PERMUTE: within every 32-column chunk, receiver 4 s + kk is stored at
// column 8 kk + s (the operand order of k_adjoint_f32).
template <typename T, bool SCALED, bool PERMUTE = false>
__global__ void k_adj_prep(int m, int mp, int nf, const double *__restrict__ d, const double *__restrict__ w,
                           const float *__restrict__ ascale, T *__restrict__ Ar, T *__restrict__ Ai,
                           T *__restrict__ Wt, T *__restrict__ As = nullptr) {
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
                const double inv = 1.0 / (double)ascale[k];
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
        if (As) As[o] = cvt<T>(re + im);
    }
}

// flags[k][eb][rb] = 1 if any weight of the 16x16 block is nonzero
__global__ void k_block_flags(int m, int nb, int nf, const double *__restrict__ w, uint8_t *__restrict__ flags) {
    const int64_t tot = (int64_t)nf * nb * nb;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    const int k = (int)(idx / ((int64_t)nb * nb));
    const int64_t rem = idx - (int64_t)k * nb * nb;
    const int eb = (int)(rem / nb), rb = (int)(rem - (int64_t)eb * nb);
    uint8_t any = 0;
    for (int i = 0; i < 16 && !any; ++i) {
        const int e = eb * 16 + i;
        if (e >= m) break;
        for (int j = 0; j < 16; ++j) {
            const int r = rb * 16 + j;
            if (r >= m) break;
            if (w[((int64_t)k * m + e) * m + r] != 0.0) {
                any = 1;
                break;
            }
        }
    }
    flags[idx] = any;
}

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

template <typename S>
__global__ void __launch_bounds__(256) k_forward16(FwdParams P, const S *__restrict__ Gr, const S *__restrict__ Gi,
                                                   const double *__restrict__ delta,
                                                   const double *__restrict__ dmax, float *__restrict__ part) {
    using V = typename MM16<S>::vec;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kk = lane >> 4;
    int te, tr;
    tri_tile(blockIdx.x, P.ntl, te, tr);
    const int split = blockIdx.y, k = blockIdx.z;
    const int64_t N = P.N;
    const S *gr = Gr + (int64_t)k * P.m * N;
    const S *gi = Gi + (int64_t)k * P.m * N;
    const int e = te * 64 + 16 * wave + row;
    const int64_t ks = (int64_t)split * P.kchunk;
    const int64_t ke = std::min<int64_t>(N, ks + P.kchunk);
    const double inv_d = dmax[0] > 0.0 ? 1.0 / dmax[0] : 0.0;
    f4 re[4], im[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) re[c] = im[c] = f4{0, 0, 0, 0};
    for (int64_t xc = ks; xc < ke; xc += 32) {
        V a_r, a_i, a_n;
        float dl[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t x = xc + 8 * kk + i;
            const bool okx = x < ke;
            dl[i] = okx ? (float)(delta[x] * inv_d) : 0.0f;
            const bool ok = okx && e < P.m;
            const float vr = ok ? MM16<S>::to_f(gr[(int64_t)e * N + x]) : 0.0f;
            const float vi = ok ? MM16<S>::to_f(gi[(int64_t)e * N + x]) : 0.0f;
            a_r[i] = MM16<S>::from_f(vr);
            a_i[i] = MM16<S>::from_f(vi);
            a_n[i] = MM16<S>::from_f(-vi);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int r = tr * 64 + 16 * c + row;
            V b_r, b_i;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int64_t x = xc + 8 * kk + i;
                const bool ok = (x < ke) && (r < P.m);
                const float vr = ok ? MM16<S>::to_f(gr[(int64_t)r * N + x]) : 0.0f;
                const float vi = ok ? MM16<S>::to_f(gi[(int64_t)r * N + x]) : 0.0f;
                b_r[i] = MM16<S>::from_f(vr * dl[i]);
                b_i[i] = MM16<S>::from_f(vi * dl[i]);
            }
            re[c] = MM16<S>::mma(a_r, b_r, re[c]);
            re[c] = MM16<S>::mma(a_n, b_i, re[c]);
            im[c] = MM16<S>::mma(a_r, b_i, im[c]);
            im[c] = MM16<S>::mma(a_i, b_r, im[c]);
        }
    }
    float *pp = part + ((int64_t)split * P.nf + k) * P.mp * P.mp * 2;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int r = tr * 64 + 16 * c + row;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ee = te * 64 + 16 * wave + 4 * kk + i;
            const int64_t o = ((int64_t)ee * P.mp + r) * 2;
            pp[o] = re[c][i];
            pp[o + 1] = im[c][i];
        }
    }
}

// d[k][e][r] = c_k * sum_split part (fixed order), read from the upper triangle.
template <typename T>
__global__ void k_forward_reduce(FwdParams P, const T *__restrict__ part, const float *__restrict__ gscale,
                                 const double *__restrict__ dmax, double *__restrict__ d) {
    const int64_t mm = (int64_t)P.m * P.m;
    const int64_t tot = mm * P.nf;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    const int k = (int)(idx / mm);
    const int64_t rem = idx - (int64_t)k * mm;
    int e = (int)(rem / P.m), r = (int)(rem - (int64_t)e * P.m);
    // d is symmetric: both (e, r) and (r, e) take the upper-triangle element
    if (e > r) {
        const int t = e;
        e = r;
        r = t;
    }
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < P.nsplit; ++s) {
        const T *pp = part + ((int64_t)s * P.nf + k) * P.mp * P.mp * 2 + ((int64_t)e * P.mp + r) * 2;
        sr += (double)pp[0];
        si += (double)pp[1];
    }
    double c = P.cg[k];
    if (gscale) {
        const double g = (double)gscale[k];
        c *= g * g;
    }
    if (dmax) c *= dmax[0];
    d[2 * idx] = sr * c;
    d[2 * idx + 1] = si * c;
}

__global__ void k_absmax_f64(const double *__restrict__ v, int64_t n, double *__restrict__ out) {
    __shared__ double sh[1024];
    double best = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) best = fmax(best, fabs(v[i]));
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// ------------------------------------------------------------------ FP32, LDS-staged
// Backprojection.  The workgroup owns 64 pixels; its four waves are 2
// (emitter halves) x 2 (pixel halves), each computing 32 e x 32 px of Y, Z
// per chunk of 64 emitters.  Receivers are consumed 32 at a time: the G tile
// [32 r][64 px] is staged in LDS, double buffered, with a row stride of 80
// floats so the four lane groups (rows 4 s + kk) fall on disjoint banks.  A
// is stored k-permuted, so a lane's eight A values of a chunk are two float4
// loads (served from L2: A is shared by every workgroup).
constexpr int kAdjNT = 64, kAdjKC = 32, kAdjLD = 80;

__device__ __forceinline__ void adj_stage_load(const float *__restrict__ gr, const float *__restrict__ gi, int m,
                                               int64_t N, int rc, int64_t x0, bool vec, f4 (&v)[4]) {
    const int t = threadIdx.x;
    const int rr = t >> 3, c4 = (t & 7) * 4;
    const int r = rc + rr;
    if (vec) {
        if (r < m) {
            const float *pr = gr + (int64_t)r * N + x0 + c4;
            const float *pi = gi + (int64_t)r * N + x0 + c4;
            v[0] = *reinterpret_cast<const f4 *>(pr);
            v[1] = *reinterpret_cast<const f4 *>(pr + 32);
            v[2] = *reinterpret_cast<const f4 *>(pi);
            v[3] = *reinterpret_cast<const f4 *>(pi + 32);
        } else {
            v[0] = v[1] = v[2] = v[3] = f4{0, 0, 0, 0};
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t xa = x0 + c4 + q, xb = xa + 32;
            const bool oka = r < m && xa < N, okb = r < m && xb < N;
            v[0][q] = oka ? gr[(int64_t)r * N + xa] : 0.0f;
            v[1][q] = okb ? gr[(int64_t)r * N + xb] : 0.0f;
            v[2][q] = oka ? gi[(int64_t)r * N + xa] : 0.0f;
            v[3][q] = okb ? gi[(int64_t)r * N + xb] : 0.0f;
        }
    }
}

__device__ __forceinline__ void adj_stage_store(float (*sB)[kAdjKC][kAdjLD], const f4 (&v)[4]) {
    const int t = threadIdx.x;
    const int rr = t >> 3, c4 = (t & 7) * 4;
    *reinterpret_cast<f4 *>(&sB[0][rr][c4]) = v[0];
    *reinterpret_cast<f4 *>(&sB[0][rr][c4 + 32]) = v[1];
    *reinterpret_cast<f4 *>(&sB[1][rr][c4]) = v[2];
    *reinterpret_cast<f4 *>(&sB[1][rr][c4 + 32]) = v[3];
}

// NB row blocks starting at b0.  The complex product Y = A conj(G) uses
// three real products, P1 = Ar Gr, P2 = Ai Gi, P3 = (Ar + Ai)(Gr - Gi), so
// Yr = P1 + P2 and Yi = P3 - P1 + P2; with the Hessian term Z = W |G|^2 that
// is four MFMAs per block and step, each on a different accumulator.
template <int NB>
__device__ __forceinline__ void adj_mma_steps(const f4 (&va)[2][2], const f4 (&vi)[2][2], const f4 (&vs)[2][2],
                                              const f4 (&vw)[2][2], float (*sBr)[kAdjLD], float (*sBi)[kAdjLD],
                                              int kk, int xc0, f4 (&p1)[2][2], f4 (&p2)[2][2], f4 (&p3)[2][2],
                                              f4 (&z)[2][2], int b0) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        // B fragments for four steps at a time (one LDS wait per half chunk)
        float br[4][2], bi[4][2];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                br[q4][cb] = sBr[4 * (4 * half + q4) + kk][xc0 + 16 * cb];
                bi[q4][cb] = sBi[4 * (4 * half + q4) + kk][xc0 + 16 * cb];
            }
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) {
        const int s8 = 4 * half + q4;
        float b2[2], bd[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            b2[cb] = br[q4][cb] * br[q4][cb] + bi[q4][cb] * bi[q4][cb];
            bd[cb] = br[q4][cb] - bi[q4][cb];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int b = b0 + q;
            const float a_r = va[b][s8 >> 2][s8 & 3], a_i = vi[b][s8 >> 2][s8 & 3];
            const float a_s = vs[b][s8 >> 2][s8 & 3], a_w = vw[b][s8 >> 2][s8 & 3];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                p1[b][cb] = MM<float>::mma(a_r, br[q4][cb], p1[b][cb]);
                p2[b][cb] = MM<float>::mma(a_i, bi[q4][cb], p2[b][cb]);
                p3[b][cb] = MM<float>::mma(a_s, bd[cb], p3[b][cb]);
                z[b][cb] = MM<float>::mma(a_w, b2[cb], z[b][cb]);
            }
        }
    }
    }
}

__global__ void __launch_bounds__(256, 2) k_adjoint_f32(AdjParams P, const float *__restrict__ Gr,
                                                        const float *__restrict__ Gi, const float *__restrict__ Ar,
                                                        const float *__restrict__ Ai, const float *__restrict__ As,
                                                        const float *__restrict__ Wt,
                                                        const uint8_t *__restrict__ flags, double *__restrict__ pg,
                                                        double *__restrict__ ph) {
    __shared__ float sB[2][2][kAdjKC][kAdjLD];
    __shared__ double sred[2][2][kAdjNT];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const int row = lane & 15, kk = lane >> 4;
    const int we = wave >> 1, wp = wave & 1;
    const int64_t N = P.N;
    const int64_t x0 = (int64_t)blockIdx.x * kAdjNT;
    const bool vec = ((N & 3) == 0) && (x0 + kAdjNT <= N);
    const int nch = P.mp / kAdjKC;
    double gacc[2] = {0.0, 0.0}, hacc[2] = {0.0, 0.0};

    {
        const int k = blockIdx.y;   // one frequency per workgroup (finer work units)
        const float *gr = Gr + (int64_t)k * P.m * N;
        const float *gi = Gi + (int64_t)k * P.m * N;
        const float *ar = Ar + (int64_t)k * P.mp * P.mp;
        const float *ai = Ai + (int64_t)k * P.mp * P.mp;
        const float *as = As + (int64_t)k * P.mp * P.mp;
        const float *wt = Wt + (int64_t)k * P.mp * P.mp;
        const uint8_t *fl = flags + (int64_t)k * P.nb * P.nb;
        float gp[2] = {0.0f, 0.0f}, hp[2] = {0.0f, 0.0f};
        for (int ec = 0; ec < P.mp; ec += 64) {
            f4 p1[2][2], p2[2][2], p3[2][2], z[2][2];
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) p1[b][c] = p2[b][c] = p3[b][c] = z[b][c] = f4{0, 0, 0, 0};
            f4 stg[4];
            adj_stage_load(gr, gi, P.m, N, 0, x0, vec, stg);
            adj_stage_store(sB[0], stg);
            __syncthreads();
            for (int c = 0; c < nch; ++c) {
                const int rc = c * kAdjKC, buf = c & 1;
                if (c + 1 < nch) adj_stage_load(gr, gi, P.m, N, rc + kAdjKC, x0, vec, stg);
                bool on[2];
                f4 va[2][2], vi[2][2], vs[2][2], vw[2][2];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int eb = (ec >> 4) + 2 * we + b;
                    on[b] = (eb < P.nb) && (fl[eb * P.nb + (rc >> 4)] | fl[eb * P.nb + (rc >> 4) + 1]);
                }
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    if (on[0] || on[1]) {
                        const int64_t off = (int64_t)(ec + 32 * we + 16 * b + row) * P.mp + rc + 8 * kk;
                        va[b][0] = *reinterpret_cast<const f4 *>(ar + off);
                        va[b][1] = *reinterpret_cast<const f4 *>(ar + off + 4);
                        vi[b][0] = *reinterpret_cast<const f4 *>(ai + off);
                        vi[b][1] = *reinterpret_cast<const f4 *>(ai + off + 4);
                        vs[b][0] = *reinterpret_cast<const f4 *>(as + off);
                        vs[b][1] = *reinterpret_cast<const f4 *>(as + off + 4);
                        vw[b][0] = *reinterpret_cast<const f4 *>(wt + off);
                        vw[b][1] = *reinterpret_cast<const f4 *>(wt + off + 4);
                    }
                }
                if (on[0] || on[1]) {
                    // a block that is off holds exact zeros in A and W, so it
                    // may be computed along with the other one
                    adj_mma_steps<2>(va, vi, vs, vw, sB[buf][0], sB[buf][1], kk, 32 * wp + row, p1, p2, p3, z, 0);
                }
                if (c + 1 < nch) adj_stage_store(sB[buf ^ 1], stg);
                __syncthreads();
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
                        hp[cb] += (ge_r * ge_r + ge_i * ge_i) * z[b][cb][i];
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
            pg[(int64_t)blockIdx.y * N + x] = sred[0][0][tid] + sred[1][0][tid];
            ph[(int64_t)blockIdx.y * N + x] = sred[0][1][tid] + sred[1][1][tid];
        }
    }
}

// grad += sum_k pg[k], hd += sum_k ph[k] in frequency order.
__global__ void k_adj_sum(int64_t N, int nf, const double *__restrict__ pg, const double *__restrict__ ph,
                          double *__restrict__ grad, double *__restrict__ hd) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    double g = 0.0, h = 0.0;
    for (int k = 0; k < nf; ++k) {
        g += pg[(int64_t)k * N + x];
        h += ph[(int64_t)k * N + x];
    }
    grad[x] += g;
    if (hd) hd[x] += h;
}

// Forward.  A 64 x 64 (e, r) output tile per workgroup (upper triangle only)
// over a split of the pixels; waves are 2 x 2, each 32 e x 32 r.  Pixels are
// consumed 32 at a time: G_e and G_r delta for the tile's rows are staged in
// LDS as [row][32 px] (stride 36: conflict-free b128 reads), double
// buffered; a lane reads its eight k values of a row as two b128 reads.
constexpr int kFwdKC = 32, kFwdLD = 36;

struct FwdStage {
    f4 ar[2], ai[2], br[2], bi[2];
};

__device__ __forceinline__ void fwd_stage_load(const float *__restrict__ gr, const float *__restrict__ gi,
                                               const double *__restrict__ delta, int m, int64_t N, int e_row,
                                               int r_row, int64_t xc, int64_t ke, bool vec, FwdStage &v) {
    const int c8 = (threadIdx.x & 3) * 8;
    const int64_t xs = xc + c8;
    if (vec) {
        double dl[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) dl[q] = delta[xs + q];
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
            f4 t0 = *reinterpret_cast<const f4 *>(pr), t1 = *reinterpret_cast<const f4 *>(pr + 4);
            f4 u0 = *reinterpret_cast<const f4 *>(pi), u1 = *reinterpret_cast<const f4 *>(pi + 4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v.br[0][q] = t0[q] * (float)dl[q];
                v.br[1][q] = t1[q] * (float)dl[q + 4];
                v.bi[0][q] = u0[q] * (float)dl[q];
                v.bi[1][q] = u1[q] * (float)dl[q + 4];
            }
        } else {
            v.br[0] = v.br[1] = v.bi[0] = v.bi[1] = f4{0, 0, 0, 0};
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t x = xs + q;
            const bool okx = x < ke;
            const float dl = okx ? (float)delta[x] : 0.0f;
            const bool oka = okx && e_row < m, okb = okx && r_row < m;
            v.ar[q >> 2][q & 3] = oka ? gr[(int64_t)e_row * N + x] : 0.0f;
            v.ai[q >> 2][q & 3] = oka ? gi[(int64_t)e_row * N + x] : 0.0f;
            v.br[q >> 2][q & 3] = okb ? gr[(int64_t)r_row * N + x] * dl : 0.0f;
            v.bi[q >> 2][q & 3] = okb ? gi[(int64_t)r_row * N + x] * dl : 0.0f;
        }
    }
}

__global__ void __launch_bounds__(256, 2) k_forward_f32(FwdParams P, const float *__restrict__ Gr,
                                                        const float *__restrict__ Gi,
                                                        const double *__restrict__ delta, float *__restrict__ part) {
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
    // (a + ib)(c + id) with three real products: P1 = ac, P2 = bd,
    // P3 = (a + b)(c + d); re = P1 - P2, im = P3 - P1 - P2
    f4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) p1[b][c] = p2[b][c] = p3[b][c] = f4{0, 0, 0, 0};
    FwdStage stg;
    auto vec_ok = [&](int64_t xc) { return ((N & 3) == 0) && (xc + kFwdKC <= ke); };
    auto store = [&](int buf) {
        *reinterpret_cast<f4 *>(&sA[buf][0][srow][c8]) = stg.ar[0];
        *reinterpret_cast<f4 *>(&sA[buf][0][srow][c8 + 4]) = stg.ar[1];
        *reinterpret_cast<f4 *>(&sA[buf][1][srow][c8]) = stg.ai[0];
        *reinterpret_cast<f4 *>(&sA[buf][1][srow][c8 + 4]) = stg.ai[1];
        *reinterpret_cast<f4 *>(&sBm[buf][0][srow][c8]) = stg.br[0];
        *reinterpret_cast<f4 *>(&sBm[buf][0][srow][c8 + 4]) = stg.br[1];
        *reinterpret_cast<f4 *>(&sBm[buf][1][srow][c8]) = stg.bi[0];
        *reinterpret_cast<f4 *>(&sBm[buf][1][srow][c8 + 4]) = stg.bi[1];
    };
    if (nch > 0) {
        fwd_stage_load(gr, gi, delta, P.m, N, e_row, r_row, ks, ke, vec_ok(ks), stg);
        store(0);
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        const int64_t xn = ks + (int64_t)(c + 1) * kFwdKC;
        if (c + 1 < nch) fwd_stage_load(gr, gi, delta, P.m, N, e_row, r_row, xn, ke, vec_ok(xn), stg);
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
        if (c + 1 < nch) store(buf ^ 1);
        __syncthreads();
    }
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

}  // namespace

// ---------------------------------------------------------------- host side
// Compute units of the current device (cached per device; 256 on MI355X).
static int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

// rows/columns of the adjoint operands are padded to a multiple of 32
static int pad_m(int m) { return (m + 31) / 32 * 32; }

AdjParams adj_params(const rb_geometry *g, const double *freqs, int nf) {
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
    void *Ar, *Ai, *Wt, *As;
    uint8_t *flags;
    float *ascale;
    double *pg, *ph;  // per-frequency partials of the f32 backprojection
};

static AdjWs carve_adj(Carver &c, const rb_geometry *g, int nf, rb_dtype dt) {
    const int mp = pad_m(g->m);
    const size_t per = (size_t)nf * mp * mp;
    const size_t es = dt == RB_F64 ? 8 : (dt == RB_F32 ? 4 : 2);
    AdjWs w;
    w.Ar = c.take<char>(per * es);
    w.Ai = c.take<char>(per * es);
    w.Wt = c.take<char>(per * es);
    w.As = c.take<char>(per * es);
    w.flags = c.take<uint8_t>((size_t)nf * (mp / 16) * (mp / 16));
    w.ascale = c.take<float>(RB_MAX_NF);
    w.pg = c.take<double>((size_t)nf * g->nx * g->ny);
    w.ph = c.take<double>((size_t)nf * g->nx * g->ny);
    return w;
}

size_t adjoint_workspace_bytes(const rb_geometry *g, int nf, rb_dtype dt) {
    Carver c(nullptr, 0);
    carve_adj(c, g, nf, dt);
    return c.used + 256;
}

rb_status adjoint_impl(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                       rb_dtype dt, const double *freqs, int nf, const double *d_res, const double *w_data,
                       double *grad, double *hdiag, void *ws, size_t ws_bytes, hipStream_t st) {
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
    if (scaled) {
        k_adj_absmax<<<nf, 256, 0, st>>>(g->m, d_res, w_data, w.ascale);
        RB_LAUNCHED();
    }
    switch (dt) {
        case RB_F64:
            k_adj_prep<double, false><<<bp, 256, 0, st>>>(g->m, P.mp, nf, d_res, w_data, nullptr, (double *)w.Ar,
                                                          (double *)w.Ai, (double *)w.Wt);
            break;
        case RB_F32:
            k_adj_prep<float, false, true><<<bp, 256, 0, st>>>(g->m, P.mp, nf, d_res, w_data, nullptr,
                                                               (float *)w.Ar, (float *)w.Ai, (float *)w.Wt,
                                                               (float *)w.As);
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
    const int64_t nfl = (int64_t)nf * P.nb * P.nb;
    k_block_flags<<<blocks_for(nfl, 256), 256, 0, st>>>(g->m, P.nb, nf, w_data, w.flags);
    RB_LAUNCHED();
    switch (dt) {
        case RB_F64: {
            const unsigned nb = blocks_for(P.N, 64 * 2);
            k_adjoint<double, 2, 2><<<nb, 256, 0, st>>>(P, (const double *)G_re, (const double *)G_im,
                                                        (const double *)w.Ar, (const double *)w.Ai,
                                                        (const double *)w.Wt, w.flags, grad, hdiag);
            break;
        }
        case RB_F32: {
            dim3 ga(blocks_for(P.N, kAdjNT), nf);
            k_adjoint_f32<<<ga, 256, 0, st>>>(P, (const float *)G_re, (const float *)G_im, (const float *)w.Ar,
                                              (const float *)w.Ai, (const float *)w.As, (const float *)w.Wt, w.flags,
                                              w.pg, w.ph);
            RB_LAUNCHED();
            k_adj_sum<<<blocks_for(P.N, 256), 256, 0, st>>>(P.N, nf, w.pg, w.ph, grad, hdiag);
            break;
        }
        case RB_BF16: {
            const unsigned nb = blocks_for(P.N, 64 * 2);
            k_adjoint16<__hip_bfloat16, 4, 2><<<nb, 256, 0, st>>>(
                P, (const __hip_bfloat16 *)G_re, (const __hip_bfloat16 *)G_im, (const __hip_bfloat16 *)w.Ar,
                (const __hip_bfloat16 *)w.Ai, (const __hip_bfloat16 *)w.Wt, w.flags, gscale, w.ascale, grad, hdiag);
            break;
        }
        case RB_F16: {
            const unsigned nb = blocks_for(P.N, 64 * 2);
            k_adjoint16<__half, 4, 2><<<nb, 256, 0, st>>>(P, (const __half *)G_re, (const __half *)G_im,
                                                          (const __half *)w.Ar, (const __half *)w.Ai,
                                                          (const __half *)w.Wt, w.flags, gscale, w.ascale, grad,
                                                          hdiag);
            break;
        }
    }
    RB_LAUNCHED();
    return RB_OK;
}

FwdParams fwd_params(const rb_geometry *g, const double *freqs, int nf, rb_dtype dt) {
    FwdParams P;
    P.m = g->m;
    P.mp = (g->m + 63) / 64 * 64;
    P.N = (int64_t)g->nx * g->ny;
    P.nf = nf;
    P.ntl = P.mp / 64;
    const int ntri = P.ntl * (P.ntl + 1) / 2;
    // about four rounds of resident workgroups (two per CU), rounded down so
    // the last round is full
    const int want = 4 * 2 * device_cus();
    int nsplit = std::max(1, want / (ntri * nf));
    const int kq = (dt == RB_BF16 || dt == RB_F16) ? 32 : 16;
    int64_t kchunk = (P.N + nsplit - 1) / nsplit;
    kchunk = (kchunk + kq - 1) / kq * kq;
    if (kchunk < kq) kchunk = kq;
    nsplit = (int)((P.N + kchunk - 1) / kchunk);
    P.nsplit = nsplit;
    P.kchunk = kchunk;
    P.ntri = ntri;
    const double dA = g->h * g->h;
    for (int k = 0; k < nf; ++k) {
        const double om = 2.0 * M_PI * (freqs ? freqs[k] : 1.0);
        P.cg[k] = om * om * dA;
    }
    return P;
}

size_t forward_workspace_bytes(const rb_geometry *g, int nf, rb_dtype dt) {
    FwdParams P = fwd_params(g, nullptr, nf, dt);
    const size_t es = dt == RB_F64 ? 8 : 4;
    return (size_t)P.nsplit * nf * P.mp * P.mp * 2 * es + 2 * 256 + 256;
}

rb_status forward_impl(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                       rb_dtype dt, const double *freqs, int nf, const double *delta, double *d_out, void *ws,
                       size_t ws_bytes, hipStream_t st) {
    if (ws_bytes < forward_workspace_bytes(g, nf, dt)) {
        set_error("forward workspace too small: need %zu bytes", forward_workspace_bytes(g, nf, dt));
        return RB_ENOMEM;
    }
    FwdParams P = fwd_params(g, freqs, nf, dt);
    Carver c(ws, ws_bytes);
    double *dmax = c.take<double>(1);
    const size_t es = dt == RB_F64 ? 8 : 4;
    void *part = c.take<char>((size_t)P.nsplit * nf * P.mp * P.mp * 2 * es);
    dim3 grid(P.ntri, P.nsplit, nf);
    const int64_t tot = (int64_t)nf * P.m * P.m;
    switch (dt) {
        case RB_F64:
            k_forward<double><<<grid, 256, 0, st>>>(P, (const double *)G_re, (const double *)G_im, delta,
                                                    (double *)part);
            RB_LAUNCHED();
            k_forward_reduce<double><<<blocks_for(tot, 256), 256, 0, st>>>(P, (const double *)part, nullptr,
                                                                           nullptr, d_out);
            break;
        case RB_F32:
            k_forward_f32<<<grid, 256, 0, st>>>(P, (const float *)G_re, (const float *)G_im, delta, (float *)part);
            RB_LAUNCHED();
            k_forward_reduce<float><<<blocks_for(tot, 256), 256, 0, st>>>(P, (const float *)part, gscale, nullptr,
                                                                          d_out);
            break;
        case RB_BF16:
        case RB_F16:
            k_absmax_f64<<<1, 1024, 0, st>>>(delta, P.N, dmax);
            RB_LAUNCHED();
            if (dt == RB_BF16)
                k_forward16<__hip_bfloat16><<<grid, 256, 0, st>>>(P, (const __hip_bfloat16 *)G_re,
                                                                  (const __hip_bfloat16 *)G_im, delta, dmax,
                                                                  (float *)part);
            else
                k_forward16<__half><<<grid, 256, 0, st>>>(P, (const __half *)G_re, (const __half *)G_im, delta,
                                                          dmax, (float *)part);
            RB_LAUNCHED();
            k_forward_reduce<float><<<blocks_for(tot, 256), 256, 0, st>>>(P, (const float *)part, gscale, dmax,
                                                                          d_out);
            break;
    }
    RB_LAUNCHED();
    return RB_OK;
}

static rb_status check_contraction(const rb_geometry *g, const void *G_re, const void *G_im, const float *scale,
                                   rb_dtype dt, const double *freqs, int32_t nf) {
    RB_TRY(check_geometry(g));
    RB_TRY(check_freqs(freqs, nf));
    RB_CHECK_ARG(dt >= RB_F64 && dt <= RB_F16, "unknown dtype %d", (int)dt);
    RB_CHECK_ARG(G_re && G_im, "G_re/G_im are NULL");
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

}  // extern "C"
