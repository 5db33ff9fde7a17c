// mfma_fft.hpp - radix-16 Stockham stages as complex 16 x 16 DFT products on
// the gfx950 matrix cores, with split-BF16 operands and FP32 accumulation.
//
// A radix-16 butterfly y_s = sum_r e^{-2 pi i r s / 16} u_r is one column of
// a real product D = A B: the 16 outputs' real parts (and, with a second
// matrix, their imaginary parts) are rows m of A (16 x 32), the inputs are
// column n of B (32 x 16) with real and imaginary parts interleaved along K:
//   Re y_m = sum_r ( c u_r.re + s u_r.im ),  Im y_m = sum_r ( -s u_r.re + c u_r.im ),
//   c = cos(2 pi m r / 16), s = sin(2 pi m r / 16).
// One v_mfma_f32_16x16x32_bf16 therefore runs 16 butterflies.  Each operand
// x is split as x = hi + lo with hi = bf16(x), lo = bf16(x - hi), and
// A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi (the lo-lo term is below the FP32
// accumulation's resolution), so a radix-16 stage costs six MFMAs per 16
// butterflies and keeps about 16 significant bits per product.
//
// Lane layout of the 16x16x32 BF16 MFMA (64 lanes, g = lane / 16,
// n = lane % 16): A[m = n][k = 8 g + i] and B[k = 8 g + i][col = n] for the
// eight operand elements i; D[row = 4 g + i][col = n] for the four results.
// So lane (g, n) supplies inputs r = 4g .. 4g+3 of butterfly n and receives
// its outputs s = 4g .. 4g+3.
#pragma once
#include "fft_core.hpp"

namespace lctk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// cos(2 pi q / 16)
__device__ __forceinline__ float cos16(int q)
{
    q &= 15;
    if (q > 8)
        q = 16 - q;
    const float a = q == 0 ? 1.0f
                  : q == 1 ? 0.92387953251128675613f
                  : q == 2 ? 0.70710678118654752440f
                  : q == 3 ? 0.38268343236508977173f
                  : 0.0f;
    const float b = q == 8 ? 1.0f
                  : q == 7 ? 0.92387953251128675613f
                  : q == 6 ? 0.70710678118654752440f
                  : q == 5 ? 0.38268343236508977173f
                  : 0.0f;
    return q <= 4 ? a : -b;
}

// This lane's fragments of the real-part and imaginary-part DFT matrices.
struct Dft16Frag {
    bf16x8 re_hi, re_lo, im_hi, im_lo;
};

__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// The same split for the four complex operands of a lane, the real and
// imaginary parts of each rounded as one pair (one packed conversion for the
// two hi parts and one for the two lo parts).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void split4_bf16(const C<float> *u, bf16x8 &bh, bf16x8 &bl)
{
    u32x4v h4, l4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const f32x2 x = {u[i].x, u[i].y};
        const bf16x2 h = __builtin_convertvector(x, bf16x2);
        const bf16x2 l = __builtin_convertvector(x - __builtin_convertvector(h, f32x2), bf16x2);
        h4[i] = __builtin_bit_cast(unsigned int, h);
        l4[i] = __builtin_bit_cast(unsigned int, l);
    }
    bh = __builtin_bit_cast(bf16x8, h4);
    bl = __builtin_bit_cast(bf16x8, l4);
}

__device__ __forceinline__ Dft16Frag dft16_frag(int lane)
{
    const int m = lane & 15, g = lane >> 4;
    Dft16Frag f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = 8 * g + i, r = k >> 1;
        const int q = (m * r) & 15;
        const float c = cos16(q), s = cos16(q + 12); // sin(2 pi q / 16) = cos(2 pi (q - 4) / 16)
        const float are = (k & 1) ? s : c;
        const float aim = (k & 1) ? c : -s;
        __bf16 h, l;
        split_bf16(are, h, l);
        f.re_hi[i] = h;
        f.re_lo[i] = l;
        split_bf16(aim, h, l);
        f.im_hi[i] = h;
        f.im_lo[i] = l;
    }
    return f;
}

// One radix-16 Stockham stage over every signal slot of the work-group (slot
// sl at smem + sl * P holds a length-N sequence, N a multiple of 256).  The
// N / 16 butterflies of a slot form N / 256 groups of 16; wave w takes groups
// 4w .. 4w+3 of the work-group (four groups per wave when each slot has
// N / 16 threads).  Butterfly b reads positions b + (N/16) r, applies the
// twiddle W_{16 Ns}^{(b mod Ns) r}, and its output s goes to the Stockham
// position ((b - j) 16 + j) + s Ns, j = b mod Ns.  Reads complete (barrier)
// before any write, so the stage works in place.
__device__ __forceinline__ void mfma_stage16(C<float> *smem, int P, int N, int Ns, const Dft16Frag &A)
{
    constexpr int GPW = 4;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int gps = N >> 8;
    const int N16 = N >> 4;
    const float inv = 1.0f / (float)(16 * Ns); // exact: Ns is a power of two
    C<float> y[GPW][4];
#pragma unroll
    for (int q = 0; q < GPW; ++q) {
        const int G = wave * GPW + q;
        const int sl = G / gps;
        const int b = (G - sl * gps) * 16 + n;
        const int j = b & (Ns - 1);
        const C<float> *src = smem + (size_t)sl * P;
        C<float> u[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            u[i] = src[lds_pad(b + N16 * (4 * g + i))];
        if (Ns > 1) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                u[i] = cmul(u[i], cis_turns(-(float)(j * (4 * g + i)) * inv));
        }
        bf16x8 bh, bl;
        split4_bf16(u, bh, bl);
        f32x4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
        // small terms first
        dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.re_hi, bl, dr, 0, 0, 0);
        dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.re_lo, bh, dr, 0, 0, 0);
        dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.re_hi, bh, dr, 0, 0, 0);
        di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.im_hi, bl, di, 0, 0, 0);
        di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.im_lo, bh, di, 0, 0, 0);
        di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.im_hi, bh, di, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            y[q][i] = C<float>{dr[i], di[i]};
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < GPW; ++q) {
        const int G = wave * GPW + q;
        const int sl = G / gps;
        const int b = (G - sl * gps) * 16 + n;
        const int j = b & (Ns - 1);
        C<float> *dst = smem + (size_t)sl * P;
        const int base = (b - j) * 16 + j;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            dst[lds_pad(base + (4 * g + i) * Ns)] = y[q][i];
    }
    __syncthreads();
}

// Length-N DFT of every slot with E = 16 values per thread, like fft_lds<16>
// (input and output at positions t + T e of slot sl), but with the radix-16
// stages on the matrix cores and the other stages (radix 8, 4, 2) on the
// vector units.  Requirements: N = 16 T a multiple of 256 (a power of two),
// the work-group a whole number of waves covering all slots, every thread of
// the work-group calling it.
__device__ __forceinline__ void fft_lds_mfma(C<float> *v, C<float> *smem, int sl, int t, int T, int N, int P,
                                             const Sched &sc)
{
    constexpr int E = 16;
    C<float> *lds = smem + (size_t)sl * P;
    const Dft16Frag A = dft16_frag((int)threadIdx.x & 63);
    __syncthreads(); // earlier users of LDS are done
#pragma unroll
    for (int e = 0; e < E; ++e)
        lds[lds_pad(t + T * e)] = v[e];
    __syncthreads();
    int Ns = 1;
    for (int s = 0; s < sc.nst; ++s) {
        const int rad = sc.rad[s];
        if (rad == 16) {
            mfma_stage16(smem, P, N, Ns, A);
        } else {
            // radix 8, 4 or 2 on the vector units (only these: the radix-16
            // vector code would raise the kernel's register demand)
            stage_read<E>(lds, v, t, T);
            if (rad == 8)
                stage_compute<E, 8>(v, t, T, Ns);
            else if (rad == 4)
                stage_compute<E, 4>(v, t, T, Ns);
            else
                stage_compute<E, 2>(v, t, T, Ns);
            __syncthreads();
            if (rad == 8)
                stage_write<E, 8>(lds, v, t, T, Ns);
            else if (rad == 4)
                stage_write<E, 4>(lds, v, t, T, Ns);
            else
                stage_write<E, 2>(lds, v, t, T, Ns);
            __syncthreads();
        }
        Ns *= rad;
    }
    stage_read<E>(lds, v, t, T);
}

} // namespace lctk
