// mfma_lct_impl.hpp - the split-BF16 matrix-core LCT for N = 4096 = 16^3
// with every stage on the matrix cores and no LDS pass outside them.
//
// One signal per work-group of 256 threads (4 waves).  The 256 butterflies
// of each radix-16 stage form 16 groups of 16; wave w takes groups 4w..4w+3
// and, in the MFMA lane layout (lane = 16 g + n), lane (g, n) of group q
// owns inputs r = 4g..4g+3 and outputs s = 4g..4g+3 of butterfly
// b = 16 (4w + q) + n.  Stage 1 reads those inputs straight from HBM
// (positions b + 256 r, pre-chirped on the way), stage 2 goes through LDS
// (mfma_stage16), and stage 3's outputs (positions b + 256 s) go straight to
// HBM with the post-chirp.  HBM sees one read and one write per sample and
// LDS two passes, as in the vector-unit kernel.
#pragma once
#include "kernels_impl.hpp"

namespace lctk {

// Radix-16 butterflies of group data u[4] (this lane's inputs r = 4g..4g+3,
// already twiddled) on the matrix cores; returns this lane's outputs
// s = 4g..4g+3.
__device__ __forceinline__ void mfma_dft16(const C<float> *u, C<float> *y, const Dft16Frag &A)
{
    bf16x8 bh, bl;
    split4_bf16(u, bh, bl);
    f32x4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
    dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.re_hi, bl, dr, 0, 0, 0);
    dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.re_lo, bh, dr, 0, 0, 0);
    dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.re_hi, bh, dr, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.im_hi, bl, di, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.im_lo, bh, di, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.im_hi, bh, di, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        y[i] = C<float>{dr[i], di[i]};
}

// Twiddles W_{16 Ns}^{j r} for r = r0 .. r0 + 3: two sine/cosine pairs and
// three products.
__device__ __forceinline__ void twiddle4(int j, int r0, int Ns, C<float> *w)
{
    const float inv = 1.0f / (float)(16 * Ns); // exact: Ns is a power of two
    w[0] = cis_turns(-(float)(j * r0) * inv);
    const C<float> w1 = cis_turns(-(float)j * inv);
#pragma unroll
    for (int i = 1; i < 4; ++i)
        w[i] = cmul(w[i - 1], w1);
}

// The chirp turns of a lane's 16 positions p(q, i) = base + 16 q + 256 i
// (group q, element i): qc n_p^2 [+ (N - 1) p / (2N)] + extra with
// n_p = 2p - N + 1 = n0 + 32 q + 512 i, so that
//   n_p^2 = n0^2 + 64 n0 q + 1024 q^2 + (1024 n0 + 32768 q) i + 262144 i^2.
// The six coefficients are reduced modulo 1 from exact integers in
// double-double (quad_turns), once per lane; per group, A_q and B_q of
// turns = A_q + i B_q + i^2 C are formed and reduced in FP64, then rounded to
// FP32, and the four values of the group are evaluated in FP32 (|i| <= 3:
// about 6e-7 turns of rounding, well inside this path's 16-bit products).
struct LaneChirp {
    double a0, a1, a2, b0, b1;
    float c;
};
__device__ __forceinline__ LaneChirp lane_chirp(double qhi, double qlo, bool with_index, int base, int N,
                                                double inv2N, double extra)
{
    const Quad qq{qhi, qlo};
    const double n0 = (double)(2 * base - N + 1);
    LaneChirp L;
    L.a0 = quad_turns(qq, n0 * n0) + extra;
    L.a1 = quad_turns(qq, 64.0 * n0);
    L.a2 = quad_turns(qq, 1024.0);
    L.b0 = quad_turns(qq, 1024.0 * n0);
    L.b1 = quad_turns(qq, 32768.0);
    L.c = (float)frac_turns(quad_turns(qq, 262144.0));
    if (with_index) {
        L.a0 += index_turns(base, N, inv2N);
        L.a1 += index_turns(16, N, inv2N);
        L.b0 += index_turns(256, N, inv2N);
    }
    L.a0 = frac_turns(L.a0);
    L.a1 = frac_turns(L.a1);
    L.a2 = frac_turns(L.a2);
    L.b0 = frac_turns(L.b0);
    L.b1 = frac_turns(L.b1);
    return L;
}
// The four chirp values of group q.
__device__ __forceinline__ void lane_chirp4(const LaneChirp &L, int q, C<float> *w)
{
    const double fq = (double)q;
    const float A = (float)frac_turns(fma(fq * fq, L.a2, fma(fq, L.a1, L.a0)));
    const float B = (float)frac_turns(fma(fq, L.b1, L.b0));
#pragma unroll
    for (int i = 0; i < 4; ++i)
        w[i] = cis_turns(__builtin_amdgcn_fractf(fmaf((float)(i * i), L.c, fmaf((float)i, B, A))));
}

template <int MODE>
// Four waves per SIMD asked of the register allocation: it then fits in 101
// VGPRs without spills (134 VGPRs and 34 AGPRs unbounded, three work-groups per
// CU), and four 34.8 KiB work-groups share a CU's LDS.
__global__ __launch_bounds__(256, 4) void k_lct_mf4096(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                     LctArgs args)
{
    constexpr int N = 4096, N16 = 256;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<float> *smem = reinterpret_cast<C<float> *>(smem_raw);
    const int64_t sig = blockIdx.x;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    const double inv2N = 0.5 / (double)N;

    double m4[4] = {0.0, 0.0, 0.0, 0.0};
    if (args.M4 != nullptr) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            m4[q] = args.M4[4 * sig + q];
    }
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(in + sig * N, (uint32_t)(N * sizeof(float2)));
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(out + sig * N, (uint32_t)(N * sizeof(float2)));

    // this lane's 16 samples: group q, element i at position b_q + 256 (4g + i)
    C<float> u[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = (4 * wave + q) * 16 + n;
        const int voff = (b + N16 * 4 * g) * (int)sizeof(float2);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            u[q][i] = Buf<float>::load(rin, voff, i * N16 * (int)sizeof(float2));
    }
    const LctConst k = args.M4 != nullptr ? lct_const_from(args.nc, m4[0], m4[1], m4[2], m4[3]) : args.k;
    const float mag = (float)k.amp_mag;

    if (k.b0) {
        // b = 0 (§1): the diagonal, no DFT (the whole work-group takes this branch)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = (4 * wave + q) * 16 + n;
            const ThreadChirp cb = seq_chirp(k.post_hi, k.post_lo, false, b + N16 * 4 * g, N16, N, inv2N, k.amp_turns);
            const int voff = (b + N16 * 4 * g) * (int)sizeof(float2);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                C<float> f = cscale(chirp_at<float>(cb, i), mag);
                Buf<float>::store(cmul(u[q][i], MODE == MODE_FWD ? f : cconj(f)), rout, voff,
                                  i * N16 * (int)sizeof(float2));
            }
        }
        return;
    }

    const Dft16Frag A = dft16_frag(lane);
    // this lane's positions: b_q + 256 (4 g + i) = base + 16 q + 256 i
    const int base = 64 * wave + n + 1024 * g;

    // stage 1 (Ns = 1): input chirp, butterflies, Stockham write b 16 + s
    const LaneChirp cin = MODE == MODE_FWD ? lane_chirp(k.pre_hi, k.pre_lo, true, base, N, inv2N, 0.0)
                                           : lane_chirp(k.post_hi, k.post_lo, true, base, N, inv2N, k.amp_turns);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = (4 * wave + q) * 16 + n;
        C<float> w[4];
        lane_chirp4(cin, q, w);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if constexpr (MODE == MODE_FWD)
                u[q][i] = cmul(u[q][i], w[i]);
            else
                u[q][i] = cscale(cmul(cconj(u[q][i]), w[i]), mag);
        }
        C<float> y[4];
        mfma_dft16(u[q], y, A);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            smem[lds_pad(b * 16 + 4 * g + i)] = y[i];
    }
    __syncthreads();

    // stage 2 (Ns = 16) through LDS
    mfma_stage16(smem, lds_elems(N), N, 16, A);

    // stage 3 (Ns = 256): read, twiddle W_4096^(b r), butterflies, output
    // chirp, store positions b + 256 s
    const LaneChirp cout = MODE == MODE_FWD ? lane_chirp(k.post_hi, k.post_lo, true, base, N, inv2N, k.amp_turns)
                                            : lane_chirp(k.pre_hi, k.pre_lo, true, base, N, inv2N, 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = (4 * wave + q) * 16 + n;
        C<float> x[4], w[4], y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            x[i] = smem[lds_pad(b + N16 * (4 * g + i))];
        twiddle4(b, 4 * g, N16, w);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            x[i] = cmul(x[i], w[i]);
        mfma_dft16(x, y, A);
        C<float> cw[4];
        lane_chirp4(cout, q, cw);
        const int voff = (b + N16 * 4 * g) * (int)sizeof(float2);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            C<float> o;
            if constexpr (MODE == MODE_FWD)
                o = cscale(cmul(y[i], cw[i]), mag);
            else
                o = cconj(cmul(y[i], cw[i]));
            Buf<float>::store(o, rout, voff, i * N16 * (int)sizeof(float2));
        }
    }
}

inline hipError_t launch_lct_mf4096_t(const void *in, void *out, const LctArgs &a, int nblocks, size_t lds,
                                      hipStream_t s)
{
    auto kern = a.mode == MODE_FWD ? k_lct_mf4096<MODE_FWD> : k_lct_mf4096<MODE_ADJ>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(256), lds, s, (const float2 *)in, (float2 *)out, a);
    return hipGetLastError();
}

} // namespace lctk
