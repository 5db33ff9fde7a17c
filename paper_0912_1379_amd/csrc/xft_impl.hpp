// xft_impl.hpp - the exact-node discrete fractional transform of eq. (tmat),
//   g = sqrt(2 pi) U^T D(z) U f,  D(z) = diag(1, z, ..., z^(N-1)),
// for a batch of signals sampled at the zeros of H_N, as two dense products on
// the matrix cores:
//   pass 1:  V[s][n] = w_n sum_k f[s][k] U[n][k],   w_n = sqrt(2 pi) z^n
//   pass 2:  g[s][j] =     sum_n V[s][n] U[n][j] = sum_n V[s][n] Ut[j][n]
// Both are C = diag-scaled (A B^T) with A complex (signals x K, interleaved)
// and B real (columns x K, K contiguous): U for pass 1, its transpose Ut for
// pass 2, so that both read B along K.  A complex row is two real rows of the
// product (real and imaginary parts), so the matrix cores see a real GEMM of
// 2 batch x N by N x N.
//
// MFMA: v_mfma_{f64,f32}_16x16x4 (D 16x16 += A 16x4 B 4x16).  Lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the results sit differently
// (both read off the device with in-bounds probes): FP32 lane l, register r
// holds D[4 (l / 16) + r][l % 16], FP64 holds D[(l / 16) + 4 r][l % 16].  A
// 16-row block holds 8 signals' real (p = 0) and imaginary (p = 1) parts, at
// row 2 s + p for FP32 and s + 8 p for FP64, so that in both cases a lane
// ends with whole complex values of two signals (XLayout).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"
#include "lct_params.hpp"
#include "mfma_fft.hpp"

namespace lctk {

template <typename R> struct XMma;
template <> struct XMma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct XMma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <typename R> struct XLayout;
template <> struct XLayout<float> {
    // row of (signal s < 8, part p) in a 16-row block
    static __device__ __forceinline__ int row(int s, int p) { return 2 * s + p; }
    // lane group g = l / 16, h < 2: signal and the registers of its parts
    static __device__ __forceinline__ int sig(int g, int h) { return 2 * g + h; }
    static constexpr int re(int h) { return 2 * h; }
    static constexpr int im(int h) { return 2 * h + 1; }
};
template <> struct XLayout<double> {
    static __device__ __forceinline__ int row(int s, int p) { return s + 8 * p; }
    static __device__ __forceinline__ int sig(int g, int h) { return g + 4 * h; }
    static constexpr int re(int h) { return h; }
    static constexpr int im(int h) { return h + 2; }
};

// Work-group tile: XS signals (2 XS product rows) x XC columns (k_xft_gemm:
// XTile<R>::C), K in steps of XK; 256 threads = 4 waves as 2 x 2, each wave
// XS rows x half the columns.  The
// launch bound asks for two work-groups per CU (at most 256 registers per
// lane): at one wave per SIMD the FP64 products stalled at every barrier.
// Measured at 4096 x 4096 against this shape: K steps of 32, and two LDS
// buffers with one barrier per step, were both slower.
constexpr int XS = 64, XC = 128, XK = 16, XPAD = 1;
constexpr int XTHREADS = 256;
constexpr int XA_LD = XK + XPAD; // LDS row stride (elements)

// Columns per work-group of k_xft_gemm: 256 for FP32 (a wave's 64 x 128
// outputs reuse each fragment read over more products), 128 for FP64 (whose
// accumulators would not fit twice the width at two work-groups per CU).
template <typename R> struct XTile {
    static constexpr int C = sizeof(R) == 4 ? 256 : 128;
};

__host__ __device__ constexpr size_t xft_lds_bytes(int esize)
{
    return (size_t)(2 * XS + (esize == 4 ? 256 : 128)) * XA_LD * esize;
}

// C[s][n] = scale[n] * sum_k A[s][k] Bm[n][k]   (scale may be null: 1)
// A: batch x K complex, Bm: Ncol x K real, C: batch x Ncol complex, all
// row-major and dense; K = Ncol = N here.
template <typename R>
__global__ __launch_bounds__(XTHREADS, 2) void k_xft_gemm(const R *__restrict__ A, const R *__restrict__ Bm,
                                                       R *__restrict__ C, const R *__restrict__ scale, int N,
                                                       int64_t batch, int ncol_tiles, int ntiles)
{
    using acc_t = typename XMma<R>::acc_t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int XCR = XTile<R>::C;
    R *As = reinterpret_cast<R *>(smem_raw); // [2 XS][XA_LD]
    R *Bs = As + 2 * XS * XA_LD;             // [XCR][XA_LD]

    // signal-major logical tiles; each XCD takes a contiguous range, so the
    // work-groups that share a signal tile share one L2
    const int tile = xcd_remap((int)blockIdx.x, ntiles);
    const int st = tile / ncol_tiles, ct = tile - st * ncol_tiles;
    const int64_t s0 = (int64_t)st * XS;
    const int n0 = ct * XCR;

    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int wrow = (wave >> 1) * XS;       // first product row of this wave (of 2 XS)
    const int wcol = (wave & 1) * (XCR / 2); // first column of this wave (of XCR)

    // global -> register staging: A as XS signals x 4 threads x AQ complex,
    // B as XCR columns x BT threads x BQ reals
    constexpr int BT = XTHREADS / XCR;
    static_assert(XS * 4 == XTHREADS && XCR * BT == XTHREADS, "staging covers the tile");
    constexpr int AQ = XK / 4, BQ = XK / BT;
    const int as_ = tid >> 2, ak = (tid & 3) * AQ;
    const int bn = tid / BT, bk = (tid % BT) * BQ;
    const bool a_live = s0 + as_ < batch;
    const bool b_live = n0 + bn < N;
    const R *arow = A + (size_t)(a_live ? s0 + as_ : 0) * 2 * (size_t)N;
    const R *brow = Bm + (size_t)(b_live ? n0 + bn : 0) * (size_t)N;

    R ra[2 * AQ], rb[BQ];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int k = k0 + ak + q;
            const bool ok = a_live && k < N;
            ra[2 * q] = ok ? arow[2 * k] : (R)0;
            ra[2 * q + 1] = ok ? arow[2 * k + 1] : (R)0;
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const int k = k0 + bk + q;
            rb[q] = (b_live && k < N) ? brow[k] : (R)0;
        }
    };
    const int arow_re = 16 * (as_ >> 3) + XLayout<R>::row(as_ & 7, 0);
    const int arow_im = 16 * (as_ >> 3) + XLayout<R>::row(as_ & 7, 1);
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            As[arow_re * XA_LD + ak + q] = ra[2 * q];
            As[arow_im * XA_LD + ak + q] = ra[2 * q + 1];
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q)
            Bs[bn * XA_LD + bk + q] = rb[q];
    };

    constexpr int RB = XS / 16, CB = XCR / 32; // 16 x 16 blocks per wave
    acc_t acc[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
            acc[i][j] = acc_t{(R)0, (R)0, (R)0, (R)0};

    fetch(0);
    for (int k0 = 0; k0 < N; k0 += XK) {
        __syncthreads(); // the previous step's reads of LDS are done
        stash();
        __syncthreads();
        if (k0 + XK < N)
            fetch(k0 + XK); // next tile in flight during the products
#pragma unroll
        for (int kk = 0; kk < XK; kk += 4) {
            R a[RB], b[CB];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                a[i] = As[(wrow + 16 * i + li) * XA_LD + kk + lg];
#pragma unroll
            for (int j = 0; j < CB; ++j)
                b[j] = Bs[(wcol + 16 * j + li) * XA_LD + kk + lg];
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < CB; ++j)
                    acc[i][j] = XMma<R>::mma(a[i], b[j], acc[i][j]);
        }
    }

    // epilogue: block i holds signals wrow / 2 + 8 i + (0 .. 7); this lane
    // has two of them whole; column n = n0 + wcol + 16 j + li
#pragma unroll
    for (int j = 0; j < CB; ++j) {
        const int n = n0 + wcol + 16 * j + li;
        if (n >= N)
            continue;
        R wr = (R)1, wi = (R)0;
        if (scale != nullptr) {
            wr = scale[2 * n];
            wi = scale[2 * n + 1];
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t s = s0 + wrow / 2 + 8 * i + XLayout<R>::sig(lg, h);
                if (s >= batch)
                    continue;
                const R xr = acc[i][j][XLayout<R>::re(h)], xi = acc[i][j][XLayout<R>::im(h)];
                R *dst = C + ((size_t)s * (size_t)N + (size_t)n) * 2;
                dst[0] = xr * wr - xi * wi;
                dst[1] = xr * wi + xi * wr;
            }
        }
    }
}

// Split-BF16 variant for FP32 data: every operand x is held as x = hi + lo
// with hi = bf16(x), lo = bf16(x - hi) (about 16 significant bits), and a
// 16 x 16 block accumulates A_hi B_lo + A_lo B_hi + A_hi B_hi in FP32 with
// v_mfma_f32_16x16x32_bf16 (the lo-lo term is below FP32 resolution).  Lane l
// supplies A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16], i < 8
// (16 contiguous bytes of a K-contiguous LDS row each), and receives
// D[4 (l / 16) + r][l % 16]: the FP32 row order, so the rows of a signal are
// 2 s + p as in k_xft_gemm<float>.  The signals arrive in FP32 and are split
// while staged into LDS; U is split once, at plan creation (Bh, Bl, rows
// padded to ldb, a multiple of 8, with zeros, so that they load 16 bytes at
// a time).
// Work-group tile: 64 signals x 256 columns, each wave 64 x 128 outputs as
// 4 x 8 blocks (each fragment read feeds 3 x 4 or 3 x 8 products); K in
// steps of one MFMA K block, which keeps the hi and lo tiles of A and B in
// 60 KiB of LDS, two work-groups per CU.
constexpr int XSB_C = 256;            // columns per work-group
constexpr int XSB_K = 32;             // K step
constexpr int XSB_LD = XSB_K + 8;     // LDS row stride in bf16 (80 bytes)

__host__ __device__ constexpr size_t xft_sb_lds_bytes() { return (size_t)2 * (2 * XS + XSB_C) * XSB_LD * 2; }

__global__ __launch_bounds__(XTHREADS, 2) void k_xft_gemm_sb(const float *__restrict__ A,
                                                            const __bf16 *__restrict__ Bh,
                                                            const __bf16 *__restrict__ Bl, float *__restrict__ C,
                                                            const float *__restrict__ scale, int N, int ldb,
                                                            int64_t batch, int ncol_tiles, int ntiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __bf16 *Ah = reinterpret_cast<__bf16 *>(smem_raw); // [2 XS][XSB_LD]
    __bf16 *Al = Ah + 2 * XS * XSB_LD;
    __bf16 *Bsh = Al + 2 * XS * XSB_LD; // [XSB_C][XSB_LD]
    __bf16 *Bsl = Bsh + XSB_C * XSB_LD;

    const int tile = xcd_remap((int)blockIdx.x, ntiles);
    const int st = tile / ncol_tiles, ct = tile - st * ncol_tiles;
    const int64_t s0 = (int64_t)st * XS;
    const int n0 = ct * XSB_C;

    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int wrow = (wave >> 1) * XS;
    const int wcol = (wave & 1) * (XSB_C / 2);

    // staging: A as XS signals x 4 threads x AQ complex; B as XSB_C columns
    // x BT threads x BQ values of each of Bh, Bl
    constexpr int BT = XTHREADS / XSB_C;
    static_assert(XS * 4 == XTHREADS && XSB_C * BT == XTHREADS, "staging covers the tile");
    constexpr int AQ = XSB_K / 4, BQ = XSB_K / BT;
    static_assert(AQ % 8 == 0 && BQ % 8 == 0, "16-byte chunks");
    const int as_ = tid >> 2, ak = (tid & 3) * AQ;
    const int bn = tid / BT, bk = (tid % BT) * BQ;
    const bool a_live = s0 + as_ < batch;
    const bool b_live = n0 + bn < N;
    const float *arow = A + (size_t)(a_live ? s0 + as_ : 0) * 2 * (size_t)N;
    const __bf16 *bhrow = Bh + (size_t)(b_live ? n0 + bn : 0) * (size_t)ldb;
    const __bf16 *blrow = Bl + (size_t)(b_live ? n0 + bn : 0) * (size_t)ldb;
    const int arow_re = 16 * (as_ >> 3) + XLayout<float>::row(as_ & 7, 0);
    const int arow_im = 16 * (as_ >> 3) + XLayout<float>::row(as_ & 7, 1);

    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const float2 *acx = reinterpret_cast<const float2 *>(arow);
    float2 ra[AQ];
    u32x4 rbh[BQ / 8], rbl[BQ / 8];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int k = k0 + ak + q;
            ra[q] = (a_live && k < N) ? acx[k] : float2{0.0f, 0.0f};
        }
#pragma unroll
        for (int c = 0; c < BQ / 8; ++c) {
            const int k = k0 + bk + 8 * c; // a multiple of 8: the chunk lies inside or beyond ldb
            const bool ok = b_live && k < ldb;
            rbh[c] = ok ? *reinterpret_cast<const u32x4 *>(bhrow + k) : u32x4{0u, 0u, 0u, 0u};
            rbl[c] = ok ? *reinterpret_cast<const u32x4 *>(blrow + k) : u32x4{0u, 0u, 0u, 0u};
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int c = 0; c < AQ / 8; ++c) {
            bf16x8 hr, lr, hi_, li_;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                __bf16 h, l;
                split_bf16(ra[8 * c + q].x, h, l);
                hr[q] = h;
                lr[q] = l;
                split_bf16(ra[8 * c + q].y, h, l);
                hi_[q] = h;
                li_[q] = l;
            }
            *reinterpret_cast<bf16x8 *>(Ah + arow_re * XSB_LD + ak + 8 * c) = hr;
            *reinterpret_cast<bf16x8 *>(Al + arow_re * XSB_LD + ak + 8 * c) = lr;
            *reinterpret_cast<bf16x8 *>(Ah + arow_im * XSB_LD + ak + 8 * c) = hi_;
            *reinterpret_cast<bf16x8 *>(Al + arow_im * XSB_LD + ak + 8 * c) = li_;
        }
#pragma unroll
        for (int c = 0; c < BQ / 8; ++c) {
            *reinterpret_cast<u32x4 *>(Bsh + bn * XSB_LD + bk + 8 * c) = rbh[c];
            *reinterpret_cast<u32x4 *>(Bsl + bn * XSB_LD + bk + 8 * c) = rbl[c];
        }
    };

    constexpr int RB = XS / 16, CB = XSB_C / 32;
    f32x4 acc[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    fetch(0);
    for (int k0 = 0; k0 < N; k0 += XSB_K) {
        __syncthreads();
        stash();
        __syncthreads();
        if (k0 + XSB_K < N)
            fetch(k0 + XSB_K);
#pragma unroll
        for (int kk = 0; kk < XSB_K; kk += 32) {
            bf16x8 ah[RB], al[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int off = (wrow + 16 * i + li) * XSB_LD + kk + 8 * lg;
                ah[i] = *reinterpret_cast<const bf16x8 *>(Ah + off);
                al[i] = *reinterpret_cast<const bf16x8 *>(Al + off);
            }
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const int off = (wcol + 16 * j + li) * XSB_LD + kk + 8 * lg;
                const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(Bsh + off);
                const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(Bsl + off);
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
                }
            }
        }
    }

#pragma unroll
    for (int j = 0; j < CB; ++j) {
        const int n = n0 + wcol + 16 * j + li;
        if (n >= N)
            continue;
        float wr = 1.0f, wi = 0.0f;
        if (scale != nullptr) {
            wr = scale[2 * n];
            wi = scale[2 * n + 1];
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t s = s0 + wrow / 2 + 8 * i + XLayout<float>::sig(lg, h);
                if (s >= batch)
                    continue;
                const float xr = acc[i][j][XLayout<float>::re(h)], xi = acc[i][j][XLayout<float>::im(h)];
                float *dst = C + ((size_t)s * (size_t)N + (size_t)n) * 2;
                dst[0] = xr * wr - xi * wi;
                dst[1] = xr * wi + xi * wr;
            }
        }
    }
}

// w[n] = sqrt(2 pi) z^n, n < N, by binary powering in double-double (about
// 2 log2(n) products, each with relative error near 2^-104), rounded once.
template <typename R>
__global__ void k_xft_weights(double zr, double zi, int N, R *__restrict__ w)
{
    const int n = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (n >= N)
        return;
    CDD acc{DD{1.0, 0.0}, DD{0.0, 0.0}};
    CDD base{DD{zr, 0.0}, DD{zi, 0.0}};
    for (int e = n; e > 0; e >>= 1) {
        if (e & 1)
            acc = cdd_mul(acc, base);
        if (e > 1)
            base = cdd_mul(base, base);
    }
    const DD s2pi{2.5066282746310007, -1.8328579980459167e-16}; // sqrt(2 pi), double-double
    const DD wr = dd_mul(acc.re, s2pi), wi = dd_mul(acc.im, s2pi);
    w[2 * n] = (R)(wr.hi + wr.lo);
    w[2 * n + 1] = (R)(wi.hi + wi.lo);
}

} // namespace lctk
