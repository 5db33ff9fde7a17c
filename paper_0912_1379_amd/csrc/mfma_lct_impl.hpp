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
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        __bf16 h, l;
        split_bf16(u[i].x, h, l);
        bh[2 * i] = h;
        bl[2 * i] = l;
        split_bf16(u[i].y, h, l);
        bh[2 * i + 1] = h;
        bl[2 * i + 1] = l;
    }
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

template <int MODE>
__global__ __launch_bounds__(256) void k_lct_mf4096(const float2 *__restrict__ in, float2 *__restrict__ out,
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

    // stage 1 (Ns = 1): input chirp, butterflies, Stockham write b 16 + s
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = (4 * wave + q) * 16 + n;
        const ThreadChirp c = MODE == MODE_FWD
                                  ? seq_chirp(k.pre_hi, k.pre_lo, true, b + N16 * 4 * g, N16, N, inv2N)
                                  : seq_chirp(k.post_hi, k.post_lo, true, b + N16 * 4 * g, N16, N, inv2N, k.amp_turns);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if constexpr (MODE == MODE_FWD)
                u[q][i] = cmul(u[q][i], chirp_at<float>(c, i));
            else
                u[q][i] = cscale(cmul(cconj(u[q][i]), chirp_at<float>(c, i)), mag);
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
        const ThreadChirp c = MODE == MODE_FWD
                                  ? seq_chirp(k.post_hi, k.post_lo, true, b + N16 * 4 * g, N16, N, inv2N, k.amp_turns)
                                  : seq_chirp(k.pre_hi, k.pre_lo, true, b + N16 * 4 * g, N16, N, inv2N);
        const int voff = (b + N16 * 4 * g) * (int)sizeof(float2);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            C<float> o;
            if constexpr (MODE == MODE_FWD)
                o = cscale(cmul(y[i], chirp_at<float>(c, i)), mag);
            else
                o = cconj(cmul(y[i], chirp_at<float>(c, i)));
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
