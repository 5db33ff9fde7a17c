// fourstep_impl.hpp - the discrete LCT for N beyond one work-group's LDS:
// a four-step FFT (N = N1 N2) in two passes, with the pre-chirp fused into
// the first pass's loads and the post-chirp into the second pass's stores.
//
//   pass 1: for each column n2, the length-N1 DFT over n1 of
//           u[n1 N2 + n2] (u = pre-chirped input), times the twiddle
//           W_N^(n2 k1); stored transposed: Y[n2 N1 + k1].
//   pass 2: for each k1, the length-N2 DFT over n2 of Y[n2 N1 + k1]; its
//           output k2 is DFT index j = k1 + N1 k2, stored (post-chirped) at
//           out[j] = out[k2 N1 + k1].
// Pass 2 reads and writes exactly the same positions of `out` (the slots
// k1 + N1 m, m < N2, of its own rows k1), so `out` holds the intermediate and
// no workspace is needed; the input must not alias the output.
// A signal with b = 0 (the diagonal of §1, no DFT) is finished by pass 1 and
// skipped by pass 2.
#pragma once
#include "kernels_impl.hpp"

namespace lctk {

// Pass 1.  Work-group: one signal, C consecutive columns n2_0 .. n2_0+C-1.
// Lanes run over the columns fastest, so every load instruction reads C
// consecutive samples of a row; the results go through LDS once more so that
// every store writes consecutive k1 of one transposed row.
// NFIX > 0: the column length N1 = NFIX with its compile-time radix schedule
// (constant strides and radices keep the register demand low enough for the
// 1024-thread launch bound without spills).  The 256-thread matrix-core
// instantiations ask for three waves per SIMD: 162-166 VGPRs, no spills, three
// work-groups per CU instead of two (unbounded they take about 200).
template <typename R, int E, int MODE, bool MF = false, int NFIX = 0, int LB = max_block(sizeof(R) == 8, E)>
__global__ __launch_bounds__(LB, (MF && LB == 256) ? 3 : 1) void k_fs1(
    const typename Vec<R>::T *__restrict__ in, typename Vec<R>::T *__restrict__ out, FsArgs args)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = args.N, N1 = args.N1, N2 = args.N2, Cc = args.C, T1 = args.T1;
    const int tiles = N2 / Cc;
    const int blk = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int64_t s = blk / tiles;
    const int n20 = (int)(blk - s * tiles) * Cc;
    const int tid = (int)threadIdx.x;
    const int sl = tid % Cc; // column slot
    const int t = tid / Cc;
    const int n2 = n20 + sl;
    const double inv2N = 0.5 / (double)N;

    double m4[4] = {0.0, 0.0, 0.0, 0.0};
    if (args.M4 != nullptr) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            m4[q] = args.M4[4 * s + q];
    }
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(in + s * N, (uint32_t)(N * (int64_t)sizeof(V)));
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(out + s * N, (uint32_t)(N * (int64_t)sizeof(V)));

    // element (n1 = t + T1 e, n2) at n1 N2 + n2
    C<R> v[E];
    const int voff = (t * N2 + n2) * (int)sizeof(V);
    const int sstep = T1 * N2 * (int)sizeof(V);
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = Buf<R>::load(rin, voff, e * sstep);

    const LctConst k = args.M4 != nullptr ? lct_const_from(args.nc, m4[0], m4[1], m4[2], m4[3]) : args.k;
    const R mag = (R)k.amp_mag;
    if (k.b0) {
        // b = 0 (§1): the diagonal sqrt(d) e^{i c x_i^2/(2d)} (conjugated for
        // the adjoint) on this work-group's elements i = n1 N2 + n2, written in
        // place of the transposed intermediate; pass 2 skips the signal.  One
        // signal per work-group, so the whole group returns together.
        ChirpSeq<R> c(seq_chirp(k.post_hi, k.post_lo, false, t * N2 + n2, T1 * N2, N, inv2N, k.amp_turns));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const C<R> f = cscale(c.next(), mag);
            Buf<R>::store(cmul(v[e], MODE == MODE_FWD ? f : cconj(f)), rout, voff, e * sstep);
        }
        return;
    }
    {
        ChirpSeq<R> c(MODE == MODE_FWD
                          ? seq_chirp(k.pre_hi, k.pre_lo, true, t * N2 + n2, T1 * N2, N, inv2N)
                          : seq_chirp(k.post_hi, k.post_lo, true, t * N2 + n2, T1 * N2, N, inv2N, k.amp_turns));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (MODE == MODE_FWD)
                v[e] = cmul(v[e], c.next());
            else
                v[e] = cscale(cmul(cconj(v[e]), c.next()), mag);
        }
    }

    C<R> *lds = smem + (size_t)sl * lds_elems(N1);
    if constexpr (MF)
        fft_lds_mfma(v, smem, sl, t, T1, N1, lds_elems(N1), args.sc1);
    else if constexpr (NFIX > 0)
        fft_lds_fixed<E, NFIX>(v, lds, t);
    else
        fft_lds<E>(v, lds, t, T1, args.sc1);

    // twiddle W_N^(n2 k1), k1 = t + T1 e: turns -(n2 t + e n2 T1) / N, the two
    // integer products reduced exactly modulo N (a chirp with C = 0)
    {
        const double A = -(double)umod24(n2 * t, N) / (double)N;
        const double B = -(double)umod24(n2 * T1, N) / (double)N;
        ChirpSeq<R> w(ThreadChirp{A, B, 0.0});
#pragma unroll
        for (int e = 0; e < E; ++e)
            v[e] = cmul(v[e], w.next());
    }

    // transpose through LDS: slot sl position k1  ->  lanes along k1
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
        lds[lds_pad(t + T1 * e)] = v[e];
    __syncthreads();
    const int sl2 = tid / T1;
    const int t2 = tid - sl2 * T1;
    const C<R> *l2 = smem + (size_t)sl2 * lds_elems(N1);
    const int voff2 = ((n20 + sl2) * N1 + t2) * (int)sizeof(V);
    const int sstep2 = T1 * (int)sizeof(V);
#pragma unroll
    for (int e = 0; e < E; ++e)
        Buf<R>::store(l2[lds_pad(t2 + T1 * e)], rout, voff2, e * sstep2);
}

// Pass 2.  Work-group: one signal, RR consecutive k1; lanes run over k1
// fastest, so loads and stores both touch RR consecutive samples per row.
// NFIX > 0: the row length N2 = NFIX with its compile-time radix schedule.
template <typename R, int E, int MODE, bool MF = false, int NFIX = 0, int LB = max_block(sizeof(R) == 8, E)>
__global__ __launch_bounds__(LB, (MF && LB == 256) ? 3 : 1) void k_fs2(typename Vec<R>::T *__restrict__ out,
                                                                       FsArgs args)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = args.N, N1 = args.N1, N2 = args.N2, RR = args.RR, T2 = args.T2;
    const int tiles = N1 / RR;
    const int blk = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int64_t s = blk / tiles;
    const int k10 = (int)(blk - s * tiles) * RR;
    const int tid = (int)threadIdx.x;
    const int r = tid % RR;
    const int t = tid / RR;
    const int k1 = k10 + r;
    const double inv2N = 0.5 / (double)N;

    double m4[4] = {0.0, 0.0, 0.0, 0.0};
    if (args.M4 != nullptr) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            m4[q] = args.M4[4 * s + q];
    }
    const __amdgpu_buffer_rsrc_t rio = make_rsrc(out + s * N, (uint32_t)(N * (int64_t)sizeof(V)));
    // element n2 = t + T2 e of row k1 at n2 N1 + k1; output k2 = t + T2 e at
    // k2 N1 + k1: the same slot
    const int voff = (t * N1 + k1) * (int)sizeof(V);
    const int sstep = T2 * N1 * (int)sizeof(V);
    C<R> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = Buf<R>::load(rio, voff, e * sstep);

    const LctConst k = args.M4 != nullptr ? lct_const_from(args.nc, m4[0], m4[1], m4[2], m4[3]) : args.k;
    const R mag = (R)k.amp_mag;
    if (k.b0)
        return; // pass 1 wrote the b = 0 diagonal (one signal per work-group)

    C<R> *lds = smem + (size_t)r * lds_elems(N2);
    if constexpr (MF)
        fft_lds_mfma(v, smem, r, t, T2, N2, lds_elems(N2), args.sc2);
    else if constexpr (NFIX > 0)
        fft_lds_fixed<E, NFIX>(v, lds, t);
    else
        fft_lds<E>(v, lds, t, T2, args.sc2);

    ChirpSeq<R> c(MODE == MODE_FWD ? seq_chirp(k.post_hi, k.post_lo, true, k1 + N1 * t, N1 * T2, N, inv2N, k.amp_turns)
                                   : seq_chirp(k.pre_hi, k.pre_lo, true, k1 + N1 * t, N1 * T2, N, inv2N));
#pragma unroll
    for (int e = 0; e < E; ++e) {
        C<R> y;
        if constexpr (MODE == MODE_FWD)
            y = cscale(cmul(v[e], c.next()), mag);
        else
            y = cconj(cmul(v[e], c.next()));
        Buf<R>::store(y, rio, voff, e * sstep);
    }
}

// Sub-lengths with compile-time schedules (E = 16): the four-step splits of
// the powers of two from the first two-pass length (2^14 FP64, 2^15 FP32) to
// 2^24.
#define LCT_FS_FIXED_LIST(X) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)
// Sub-lengths 3 2^k and 5 2^k of the four-step splits of such lengths, at the
// widths the planner gives them (FP32 24 / 20, FP64 12 / 10).
#define LCT_FS_FIXED3_F32(X) X(24, 192) X(24, 384) X(24, 768) X(24, 1536) X(24, 3072)
#define LCT_FS_FIXED5_F32(X) X(20, 160) X(20, 320) X(20, 640) X(20, 1280) X(20, 2560)
#define LCT_FS_FIXED3_F64(X) X(12, 96) X(12, 192) X(12, 384) X(12, 768) X(12, 1536)
#define LCT_FS_FIXED5_F64(X) X(10, 80) X(10, 160) X(10, 320) X(10, 640) X(10, 1280)

template <typename R, int E, bool MF = false, int NFIX = 0, int LB = max_block(sizeof(R) == 8, E)>
inline hipError_t launch_fs1_t(const void *in, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    auto kern = a.mode == MODE_FWD ? k_fs1<R, E, MODE_FWD, MF, NFIX, LB> : k_fs1<R, E, MODE_ADJ, MF, NFIX, LB>;
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, s, (const typename Vec<R>::T *)in, (typename Vec<R>::T *)out,
                       a);
    return hipGetLastError();
}

template <typename R, int E, bool MF = false, int NFIX = 0, int LB = max_block(sizeof(R) == 8, E)>
inline hipError_t launch_fs2_t(void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    auto kern = a.mode == MODE_FWD ? k_fs2<R, E, MODE_FWD, MF, NFIX, LB> : k_fs2<R, E, MODE_ADJ, MF, NFIX, LB>;
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, s, (typename Vec<R>::T *)out, a);
    return hipGetLastError();
}

} // namespace lctk
