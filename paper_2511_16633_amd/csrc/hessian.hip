// Diagonal of the Gauss-Newton Hessian (paper, Inverse Problem section,
// Eq. 10; the single-step paragraph's weights) for data weights of the form
// the inversion uses: receiver selection by circular distance (Results:
// the opposite part of the ring) with some selected pairs zeroed (Results:
// the largest values of a frequency set set to zero),
//     W_er = [d(e, r) >= dmin] - [(e, r) zeroed],
//     hd(x) = sum_k omega_k^4 h^4 sum_e g_e(x) sum_r W_er g_r(x),  g = |G|^2.
// With S = sum_r g_r and B_e = sum_{d(e,r) < dmin} g_r (the band the
// selection removes), sum_r W_er g_r = S - B_e - sum_{r zeroed for e} g_r,
// so a pixel costs O(m + zeroed pairs) instead of the O(m^2) of a dense W:
// B_e is a circular window sum that slides by one receiver per emitter.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "born.h"
#include "common.h"

namespace rb {
namespace {

template <typename T>
__device__ __forceinline__ double to_d(T v) { return (double)v; }
template <>
__device__ __forceinline__ double to_d<__hip_bfloat16>(__hip_bfloat16 v) { return (double)__bfloat162float(v); }
template <>
__device__ __forceinline__ double to_d<__half>(__half v) { return (double)__half2float(v); }

constexpr int kHbThreads = 256;

// four table values loaded together (8 bytes of a 16-bit type)
template <typename T>
struct __attribute__((aligned(4 * sizeof(T)))) Vec4 {
    T v[4];
};

struct HbParams {
    int m, nf, pb, dmin, zcap;
    int64_t N;
    double ch[RB_MAX_NF];   // omega^4 h^4
};

// A block holds PB pixels; its NT threads form NT / PB groups per pixel.
// g for the block's pixels is staged in LDS as [r][PB] values of type L,
// and every sum is taken in L: FP64 for FP64 tables, else FP32 (the
// precision of the matrix-core path).  Group q loads receivers
// r = q (mod groups) and takes emitters [m q / groups, m (q + 1) / groups);
// partial sums are combined in group order, so the result is deterministic.
// The zeroed pairs pass through LDS in chunks of 2 NT, packed as
// e << 16 | r (0xffffffff for an entry out of range), double-buffered: each
// thread loads its two entries of the next chunk into registers while the
// block works on the current one, one barrier per chunk.  With FP32 sums
// and PB a multiple of 4 (ZQ) a thread takes four pixels of a zeroed pair
// at once (one 16-byte LDS read per element instead of four 4-byte ones):
// the pairs are then packed as row offsets (e PQ) << 16 | r PQ in units of
// four pixels, an entry out of range pointing at a row of zeros after the
// m rows of g, and the partial sums of the 4 NG pair groups are combined
// per pixel in group order through the chunk buffer.  Workgroups go to the
// XCDs in contiguous pixel ranges, so the table rows of neighbouring
// workgroups (64 or 128 bytes each) share L2 lines.
template <typename T, typename L, int PB, int NT = kHbThreads>
__global__ void __launch_bounds__(NT) k_hess_band(HbParams P, const T *__restrict__ Gr,
                                                          const T *__restrict__ Gi, const float *__restrict__ gscale,
                                                          const int2 *__restrict__ zeroed,
                                                          const int *__restrict__ nzero, double *__restrict__ hd) {
    constexpr int NG = NT / PB;
    constexpr bool ZQ = PB % 4 == 0 && sizeof(L) == 4;
    constexpr int PQ = ZQ ? PB / 4 : 1;       // pixel quads per row
    extern __shared__ __align__(16) unsigned char lds_raw[];
    L *sg = reinterpret_cast<L *>(lds_raw);   // [m][PB], with ZQ one more row of zeros
    __shared__ L spart[NT];
    constexpr int ZC = 2 * NT;                // zeroed pairs per chunk
    __shared__ __align__(16) unsigned sz[2][ZC];   // two chunks of the zeroed-pair list, packed
    const int m = P.m;
    const int t = threadIdx.x;
    const int px = t % PB, grp = t / PB;
    const int64_t xb = xcd_remap(blockIdx.x, gridDim.x) * PB;   // the block's first pixel
    if (ZQ && t < PB) sg[m * PB + t] = 0;     // ordered before its readers by the barriers below
    const int64_t x = xb + px;
    const bool okx = x < P.N;
    // 16-bit tables load whole, aligned pixel quads (block-uniform; with
    // 2-byte loads the load phase was bound by instruction issue: 1024
    // elements / 1100^2 bf16, 17.8 -> 12.6 ms per 4-frequency launch, while
    // FP32 tables gained nothing and keep one pixel per thread)
    constexpr bool VQ = PB % 4 == 0 && sizeof(T) == 2;
    const bool quads = (P.N % 4 == 0) && (xb + PB <= P.N);
    const L *col = sg + px;
    const int half = P.dmin - 1;              // band: r = e + s, |s| <= half
    const bool none = 2 * half + 1 >= m;      // the band covers the ring: nothing selected
    const int e0 = (m * grp) / NG, e1 = (m * (grp + 1)) / NG;
    double total = 0.0;
    for (int k = 0; k < P.nf; ++k) {
        const T *gr = Gr + (int64_t)k * m * P.N + x;
        const T *gi = Gi + (int64_t)k * m * P.N + x;
        const L sc = gscale ? (L)gscale[k] * (L)gscale[k] : (L)1;
        L sp = 0;
        if (VQ && quads) {
            // four consecutive pixels of a row per thread (one 16- or 8-byte
            // load per array), two rows in flight; this pixel's partial sum
            // over rows grp (mod NG) is then read back from LDS
            constexpr int PQ = PB >= 4 ? PB / 4 : 1, RGN = NT / PQ;
            const int pq = t % PQ, rg = t / PQ;
            const T *qr = Gr + (int64_t)k * m * P.N + xb + 4 * pq;
            const T *qi = Gi + (int64_t)k * m * P.N + xb + 4 * pq;
            for (int r0 = rg; r0 < m; r0 += 2 * RGN) {
                Vec4<T> a[2], b[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int r = r0 + u * RGN;
                    if (r < m) {
                        a[u] = *reinterpret_cast<const Vec4<T> *>(qr + (int64_t)r * P.N);
                        b[u] = *reinterpret_cast<const Vec4<T> *>(qi + (int64_t)r * P.N);
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int r = r0 + u * RGN;
                    if (r < m) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const L va = (L)to_d(a[u].v[q]), vb = (L)to_d(b[u].v[q]);
                            sg[r * PB + 4 * pq + q] = (va * va + vb * vb) * sc;
                        }
                    }
                }
            }
            __syncthreads();
            for (int r = grp; r < m; r += NG) sp += col[r * PB];
        } else
        // eight rows in flight per thread
        for (int r0 = grp; r0 < m; r0 += 8 * NG) {
            T va[8], vb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int r = r0 + u * NG;
                const bool ok = okx && r < m;
                va[u] = ok ? gr[(int64_t)r * P.N] : T(0);
                vb[u] = ok ? gi[(int64_t)r * P.N] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int r = r0 + u * NG;
                if (r < m) {
                    const L a = (L)to_d(va[u]), b = (L)to_d(vb[u]);
                    const L v = (a * a + b * b) * sc;
                    sg[r * PB + px] = v;
                    sp += v;
                }
            }
        }
        spart[t] = sp;
        __syncthreads();
        L S = 0;
        for (int q = 0; q < NG; ++q) S += spart[q * PB + px];
        L acc = 0;
        if (!none && e0 < e1) {
            // window of e0: receivers e0 - half .. e0 + half (mod m); 2 half + 1 < m
            L B = 0;
            int ri = e0 - half;
            if (ri < 0) ri += m;
#pragma unroll 8
            for (int s = -half; s <= half; ++s) {
                B += col[ri * PB];
                if (++ri == m) ri = 0;
            }
            // slide: add e + half + 1, drop e - half
            int ra = e0 + half + 1, rd = e0 - half;
            if (ra >= m) ra -= m;
            if (rd < 0) rd += m;
#pragma unroll 4
            for (int e = e0; e < e1; ++e) {
                acc += col[e * PB] * (S - B);
                if (half >= 0) {
                    B += col[ra * PB] - col[rd * PB];
                    if (++ra == m) ra = 0;
                    if (++rd == m) rd = 0;
                }
            }
        }
        // zeroed pairs, staged through LDS two chunks at a time
        const int nz = nzero ? min(nzero[k], P.zcap) : 0;   // block-uniform
        const int2 *zk = zeroed + (int64_t)k * P.zcap;
        // (m PQ < 2^16: PB = 32 only for m <= 1024)
        const unsigned zoff = ((unsigned)(m * PQ) << 16) | (unsigned)(m * PQ);   // the row of zeros
        auto fetch = [&](int c0, unsigned (&reg)[2]) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = c0 + h * NT + t;
                reg[h] = ZQ ? zoff : 0xffffffffu;
                if (i < nz) {
                    const int2 q = zk[i];
                    if ((unsigned)q.x < (unsigned)m && (unsigned)q.y < (unsigned)m)
                        reg[h] = ZQ ? (((unsigned)(q.x * PQ) << 16) | (unsigned)(q.y * PQ))
                                    : (((unsigned)q.x << 16) | (unsigned)q.y);
                }
            }
        };
        unsigned zr[2];
        if (nz > 0) fetch(0, zr);
        // ZQ: thread (gz, pq) sums pairs gz (mod 4 NG) for pixels 4 pq .. 4 pq + 3
        const int pq = t % PQ, gz = t / PQ;
        const float4 *cq = reinterpret_cast<const float4 *>(sg) + pq;
        float4 zs = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int c0 = 0, b = 0; c0 < nz; c0 += ZC, b ^= 1) {
            sz[b][t] = zr[0];
            sz[b][NT + t] = zr[1];
            __syncthreads();   // chunk b is in LDS; the chunk read two rounds ago is done
            if (c0 + ZC < nz) fetch(c0 + ZC, zr);   // in flight while chunk b is summed
            const int cn = min(ZC, nz - c0);
            if constexpr (ZQ) {
                constexpr int NGZ = NT / PQ;
                for (int i0 = gz; i0 < cn; i0 += 4 * NGZ) {
                    float4 va[4], vb[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 + u * NGZ;
                        const unsigned q = i < cn ? sz[b][i] : zoff;
                        va[u] = cq[q >> 16];
                        vb[u] = cq[q & 0xffffu];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        zs.x += va[u].x * vb[u].x;
                        zs.y += va[u].y * vb[u].y;
                        zs.z += va[u].z * vb[u].z;
                        zs.w += va[u].w * vb[u].w;
                    }
                }
                continue;
            }
            for (int i0 = grp; i0 < cn; i0 += 8 * NG) {
                L pr[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = i0 + u * NG;
                    pr[u] = 0;
                    if (i < cn) {
                        const unsigned q = sz[b][i];
                        if (q != 0xffffffffu) pr[u] = col[(int)(q >> 16) * PB] * col[(int)(q & 0xffffu) * PB];
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc -= pr[u];
            }
        }
        __syncthreads();   // every thread has read spart, sg and sz
        if constexpr (ZQ) {
            // the 4 NG pair groups' partial sums, [gz][PB] in the chunk
            // buffer; pixel px of group grp takes groups 4 grp .. 4 grp + 3
            float *zp = reinterpret_cast<float *>(&sz[0][0]);
            if (nz > 0) {
                reinterpret_cast<float4 *>(zp)[gz * PQ + pq] = zs;
                __syncthreads();
                const float *zc = zp + 4 * grp * PB + px;
                acc -= ((zc[0] + zc[PB]) + zc[2 * PB]) + zc[3 * PB];
            }
        }
        spart[t] = acc;
        __syncthreads();
        if (grp == 0) {
            L a = 0;
            for (int q = 0; q < NG; ++q) a += spart[q * PB + px];
            total += (double)a * P.ch[k];
        }
        __syncthreads();
    }
    if (grp == 0 && okx) hd[x] += total;
}

// LDS of the [m][PB] values (and the row of zeros): within 40 KiB for
// blocks of 256 threads, 140 KiB for the wide blocks (whose static arrays
// take up to 20 KiB more)
constexpr size_t kHbLds = 40960, kHbLdsWide = 143360;
// the wide blocks: pixels and threads
constexpr int kHbWidePB = 32, kHbWideNT = 1024;

}  // namespace

rb_status hessian_band_impl(const rb_geometry *g, const void *G_re, const void *G_im, const float *gscale,
                            rb_dtype dt, const double *freqs, int nf, int dmin, const int *zeroed,
                            const int *nzero, int zcap, double *hdiag, hipStream_t st) {
    HbParams P;
    P.m = g->m;
    P.nf = nf;
    P.N = (int64_t)g->nx * g->ny;
    P.dmin = dmin;
    P.zcap = zcap;
    // pixels per block: [m][pb] values within 40 KiB.  For 256 < m <= 1024
    // and 32/16-bit tables a block of 1024 threads keeps 32 pixels (up to
    // 128 KiB of LDS): reads of a table row then span 64 or 128 bytes
    // instead of 16 or 32.
    const bool f64 = dt == RB_F64;
    const bool wide = !f64 && P.m > 256 && P.m <= 1024;
    const int pb = wide ? kHbWidePB : (f64 ? (P.m <= 256 ? 16 : (P.m <= 1024 ? 4 : 1)) : (P.m <= 256 ? 32 : (P.m <= 1024 ? 8 : 2)));
    const bool zq = !f64 && pb % 4 == 0;   // the kernel's ZQ: one more row
    const size_t lds = (size_t)(P.m + (zq ? 1 : 0)) * pb * (f64 ? sizeof(double) : sizeof(float));
    if (lds > (wide ? kHbLdsWide : kHbLds)) {
        set_error("m = %d is too large for the banded Hessian", P.m);
        return RB_EUNSUPPORTED;
    }
    P.pb = pb;
    const double dA = g->h * g->h;
    for (int k = 0; k < nf; ++k) {
        const double om = 2.0 * M_PI * freqs[k];
        const double c = om * om * dA;
        P.ch[k] = c * c;
    }
    const unsigned nb = (unsigned)((P.N + pb - 1) / pb);
    const int2 *z = reinterpret_cast<const int2 *>(zeroed);
    if (zcap == 0) nzero = nullptr;
    auto go = [&](auto tag, auto ltag, const float *gs) {
        using T = decltype(tag);
        using L = decltype(ltag);
        const T *gr = static_cast<const T *>(G_re), *gi = static_cast<const T *>(G_im);
        if (wide) {
            auto kfn = k_hess_band<T, L, kHbWidePB, kHbWideNT>;
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kfn),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kfn<<<nb, kHbWideNT, lds, st>>>(P, gr, gi, gs, z, nzero, hdiag);
            return;
        }
        switch (pb) {
            case 32: k_hess_band<T, L, 32><<<nb, kHbThreads, lds, st>>>(P, gr, gi, gs, z, nzero, hdiag); break;
            case 16: k_hess_band<T, L, 16><<<nb, kHbThreads, lds, st>>>(P, gr, gi, gs, z, nzero, hdiag); break;
            case 8: k_hess_band<T, L, 8><<<nb, kHbThreads, lds, st>>>(P, gr, gi, gs, z, nzero, hdiag); break;
            case 4: k_hess_band<T, L, 4><<<nb, kHbThreads, lds, st>>>(P, gr, gi, gs, z, nzero, hdiag); break;
            case 2: k_hess_band<T, L, 2><<<nb, kHbThreads, lds, st>>>(P, gr, gi, gs, z, nzero, hdiag); break;
            default: k_hess_band<T, L, 1><<<nb, kHbThreads, lds, st>>>(P, gr, gi, gs, z, nzero, hdiag); break;
        }
    };
    switch (dt) {
        case RB_F64: go(double(), double(), nullptr); break;
        case RB_F32: go(float(), float(), nullptr); break;
        case RB_BF16: go(__hip_bfloat16(), float(), gscale); break;
        case RB_F16: go(__half(), float(), gscale); break;
    }
    RB_LAUNCHED();
    return RB_OK;
}

}  // namespace rb

extern "C" {

rb_status rb_born_hessian_banded(const rb_geometry *g, const void *G_re, const void *G_im, const float *scale,
                                 rb_dtype dtype, const double *freqs_hz, int32_t nf, int32_t dmin,
                                 const int32_t *zeroed, const int32_t *nzero, int32_t zcap, double *hdiag,
                                 void *stream) {
    rb::clear_error();
    RB_TRY(rb::check_contraction(g, G_re, G_im, scale, dtype, freqs_hz, nf));
    RB_CHECK_ARG(hdiag != nullptr, "hdiag is NULL");
    RB_CHECK_ARG(dmin >= 0, "dmin must be >= 0");
    RB_CHECK_ARG(zcap >= 0 && (zcap == 0 || (zeroed && nzero)), "zeroed/nzero are required when zcap > 0");
    return rb::hessian_band_impl(g, G_re, G_im, scale, dtype, freqs_hz, nf, dmin, zeroed, nzero, zcap, hdiag,
                                 rb::as_stream(stream));
}

}  // extern "C"
