// frft_large_impl.hpp - the same-grid fractional transform when its length
// L = 2N convolution does not fit one work-group's LDS.
//
// g = C D IDFT(DFT(v) . DFT(t)) restricted to the first N outputs, with
// v = D f zero-padded (reversed for the Hankel form) and t the Gaussian-chirp
// Toeplitz kernel.  Each length-L DFT is a four-step FFT (L = L1 L2) in two
// passes; the workspace holds three length-L regions per signal:
//   R0: DFT(v)  (pass 1 writes it transposed, pass 2 turns it into natural order in place)
//   R1: DFT(t)  (same)
//   R2: the inverse transform's transposed intermediate
// Launches: [pass 1 of v and t] [pass 2 of v and t] [pass 1 of conj(V K)] [pass 2 -> out].
#pragma once
#include "fourstep_impl.hpp"

namespace lctk {

enum FrKind { FR_DATA = 0, FR_KERN = 1, FR_INV = 2 };

template <typename R>
__device__ __forceinline__ FrConst fr_const_of(const FrLArgs &a, int64_t s)
{
    return a.Z2 != nullptr ? fr_const(a.N, a.Z2[2 * s], a.Z2[2 * s + 1]) : a.k;
}

// Pass 1 over columns n2 of the length-L sequence (element i = n1 L2 + n2).
// blockIdx.x < batch * tiles handles the data (FR_DATA, or FR_INV when
// `inverse`), the rest the kernel sequence (FR_KERN).
template <typename R, int E>
__global__ __launch_bounds__(max_block(sizeof(R) == 8, E)) void k_frl1(
    const typename Vec<R>::T *__restrict__ in, typename Vec<R>::T *__restrict__ ws, FrLArgs a, int inverse)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = a.N, L = a.L, L1 = a.L1, L2 = a.L2, Cc = a.C, T1 = a.T1;
    const int tiles = L2 / Cc;
    int64_t b = blockIdx.x;
    int kind = inverse ? FR_INV : FR_DATA;
    if (!inverse && b >= a.batch * tiles) {
        kind = FR_KERN;
        b -= a.batch * tiles;
    }
    const int64_t s = b / tiles;
    const int n20 = (int)(b - s * tiles) * Cc;
    const int tid = (int)threadIdx.x;
    const int sl = tid % Cc;
    const int t = tid / Cc;
    const int n2 = n20 + sl;
    const FrConst k = fr_const_of<R>(a, s);
    V *R0 = ws + (size_t)s * 3 * L;
    V *R1 = R0 + L;
    V *R2 = R1 + L;

    C<R> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = (t + T1 * e) * L2 + n2;
        C<R> x = {(R)0, (R)0};
        if (kind == FR_DATA) {
            if (i < N && !k.special) {
                x = ldc<R>(in + (size_t)s * N + (k.hankel ? N - 1 - i : i));
                x = cmul(x, gauss_chirp<R>(k.dmag, k.dph_hi, k.dph_lo, nsq(i, N)));
            }
        } else if (kind == FR_KERN) {
            const int m = i <= N ? i : L - i;
            x = gauss_chirp<R>(k.kmag, k.kph_hi, k.kph_lo, (double)m * (double)m);
        } else {
            x = cconj(cmul(ldc<R>(R0 + i), ldc<R>(R1 + i)));
        }
        v[e] = x;
    }

    C<R> *lds = smem + (size_t)sl * lds_elems(L1);
    fft_lds<E>(v, lds, t, T1, a.sc1);

    {
        const double A = -(double)(((int64_t)n2 * t) % L) / (double)L;
        const double B = -(double)(((int64_t)n2 * T1) % L) / (double)L;
#pragma unroll
        for (int e = 0; e < E; ++e)
            v[e] = cmul(v[e], cis_turns_from<R>(frac_turns(fma(B, (double)e, A))));
    }

    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
        lds[lds_pad(t + T1 * e)] = v[e];
    __syncthreads();
    const int sl2 = tid / T1;
    const int t2 = tid - sl2 * T1;
    const C<R> *l2 = smem + (size_t)sl2 * lds_elems(L1);
    V *dst = kind == FR_DATA ? R0 : (kind == FR_KERN ? R1 : R2);
#pragma unroll
    for (int e = 0; e < E; ++e)
        stc<R>(dst + (size_t)(n20 + sl2) * L1 + t2 + T1 * e, l2[lds_pad(t2 + T1 * e)]);
}

// Pass 2 over rows k1 (element n2 of row k1 at n2 L1 + k1).  Forward
// (inverse == 0): regions R0 and R1 in place, blocks beyond batch * tiles
// take R1.  Inverse: reads R2 and writes the first N outputs to `out`.
template <typename R, int E>
__global__ __launch_bounds__(max_block(sizeof(R) == 8, E)) void k_frl2(
    typename Vec<R>::T *__restrict__ ws, typename Vec<R>::T *__restrict__ out, FrLArgs a, int inverse)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = a.N, L = a.L, L1 = a.L1, RR = a.RR, T2 = a.T2;
    const int tiles = L1 / RR;
    int64_t b = blockIdx.x;
    int region = inverse ? 2 : 0;
    if (!inverse && b >= a.batch * tiles) {
        region = 1;
        b -= a.batch * tiles;
    }
    const int64_t s = b / tiles;
    const int k10 = (int)(b - s * tiles) * RR;
    const int tid = (int)threadIdx.x;
    const int r = tid % RR;
    const int t = tid / RR;
    const int k1 = k10 + r;
    V *reg = ws + (size_t)s * 3 * L + (size_t)region * L;

    C<R> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = ldc<R>(reg + (size_t)(t + T2 * e) * L1 + k1);

    C<R> *lds = smem + (size_t)r * lds_elems(a.L2);
    fft_lds<E>(v, lds, t, T2, a.sc2);

    if (!inverse) {
#pragma unroll
        for (int e = 0; e < E; ++e)
            stc<R>(reg + (size_t)(t + T2 * e) * L1 + k1, v[e]);
    } else {
        const FrConst k = fr_const_of<R>(a, s);
        if (k.special)
            return;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = k1 + L1 * (t + T2 * e);
            if (j < N) {
                C<R> y = cconj(v[e]);
                y = cmul(y, gauss_chirp<R>(k.dmag, k.dph_hi, k.dph_lo, nsq(j, N)));
                y = cmul(y, C<R>{(R)k.cre, (R)k.cim});
                stc<R>(out + (size_t)s * N + j, y);
            }
        }
    }
}

// z = +-1 (continuum limits): out = sqrt(2 pi) in, or reversed.  One
// work-group per signal.
template <typename R>
__global__ void k_fr_special(const typename Vec<R>::T *__restrict__ in, typename Vec<R>::T *__restrict__ out,
                             FrLArgs a)
{
    const int64_t s = blockIdx.x;
    const FrConst k = fr_const_of<R>(a, s);
    if (!k.special)
        return;
    for (int j = threadIdx.x; j < a.N; j += blockDim.x) {
        C<R> x = ldc<R>(in + (size_t)s * a.N + (k.special == 1 ? j : a.N - 1 - j));
        stc<R>(out + (size_t)s * a.N + j, cscale(x, (R)k.cre));
    }
}

template <typename R, int E>
inline hipError_t launch_frl1_t(const void *in, void *ws, const FrLArgs &a, int inverse, int nb, int bs, size_t lds,
                                hipStream_t st)
{
    using V = typename Vec<R>::T;
    auto kern = k_frl1<R, E>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, st, (const V *)in, (V *)ws, a, inverse);
    return hipGetLastError();
}

template <typename R, int E>
inline hipError_t launch_frl2_t(void *ws, void *out, const FrLArgs &a, int inverse, int nb, int bs, size_t lds,
                                hipStream_t st)
{
    using V = typename Vec<R>::T;
    auto kern = k_frl2<R, E>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, st, (V *)ws, (V *)out, a, inverse);
    return hipGetLastError();
}

template <typename R>
inline hipError_t launch_fr_special_t(const void *in, void *out, const FrLArgs &a, hipStream_t st)
{
    using V = typename Vec<R>::T;
    hipLaunchKernelGGL(k_fr_special<R>, dim3((unsigned)a.batch), dim3(256), 0, st, (const V *)in, (V *)out, a);
    return hipGetLastError();
}

} // namespace lctk
