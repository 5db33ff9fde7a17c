// oversample_impl.hpp - the aliasing-aware LCT: the N samples on x_k are
// interpolated trigonometrically onto the grid of step h / p over the same span
// (one work-group per signal, both DFTs in LDS), the LCT of §1 runs on that
// finer grid with the scaled-grid constants (s = 1 / sqrt(p)), and the N
// outputs at the Algorithm's nodes y_j, the middle block of the p N fine
// outputs, are copied out.
#pragma once
#include "kernels_impl.hpp"

namespace lctk {

// In-LDS FFT of the register values of the first T threads (positions
// t + T e); the other threads of the work-group only take part in the
// barriers.  Same stages as fft_lds.
template <int E, typename R>
__device__ __forceinline__ void fft_lds_part(C<R> *v, C<R> *lds, int t, int T, const Sched &sc, bool active)
{
    int Ns = 1;
    for (int s = 0; s < sc.nst; ++s) {
        const int rad = sc.rad[s];
        if (active)
            run_stage<E>(rad, v, t, T, Ns);
        if (s + 1 < sc.nst) {
            __syncthreads();
            if (active)
                run_write<E>(rad, lds, v, t, T, Ns);
            __syncthreads();
            if (active)
                stage_read<E>(lds, v, t, T);
        }
        Ns *= rad;
    }
}

// One signal per work-group.  With c_n = (1/N) sum_k f_k e^{-2 pi i n k / N}
// (n = k for k < N/2, k - N above; for even N the coefficient at n = -N/2 is
// split in halves between -N/2 and +N/2), the fine samples are
//   g_m = sum_n c_n e^{-i pi n (P - 1) / (P N)} e^{2 pi i n m / (P N)},
// i.e. f's trigonometric interpolant at x_0 + (h / P)(m - (P - 1)/2).
template <typename R, int E>
__global__ __launch_bounds__(1024) void k_interp(const typename Vec<R>::T *__restrict__ in,
                                                 typename Vec<R>::T *__restrict__ out, InterpArgs a)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *lds = reinterpret_cast<C<R> *>(smem_raw);
    const int N = a.N, P = a.P, M = a.N * a.P, T = a.T, T1 = a.T1;
    const int t = (int)threadIdx.x;
    const int64_t s = blockIdx.x;
    const bool act = t < T1;
    const V *src = in + (size_t)s * N;
    V *dst = out + (size_t)s * M;

    // 1) c = DFT_N(f) / N on the first T1 threads
    C<R> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = act ? ldc<R>(src + t + T1 * e) : C<R>{(R)0, (R)0};
    fft_lds_part<E>(v, lds, t, T1, a.sc1, act);

    // 2) the zero-padded, twisted coefficients in natural order (LDS, unpadded)
    __syncthreads(); // the DFT's last exchange has been read
    for (int i = t; i < M; i += T)
        lds[i] = C<R>{(R)0, (R)0};
    __syncthreads();
    if (act) {
        const R inv = (R)1 / (R)N;
        const int64_t twoM = 2 * (int64_t)M;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + T1 * e;
            const int n = k < (N + 1) / 2 ? k : k - N; // -floor(N/2) .. ceil(N/2) - 1
            const C<R> c = cscale(v[e], inv);
            // twist e^{-i pi n (P-1) / (P N)}: -n (P-1) / (2 P N) turns, reduced exactly
            auto twisted = [&](int nn) {
                int64_t num = ((int64_t)nn * (P - 1)) % twoM;
                if (num < 0)
                    num += twoM;
                return cmul(c, cis_turns_from<R>(frac_turns(-(double)num / (double)twoM)));
            };
            if ((N & 1) == 0 && 2 * n == -N) {
                // Nyquist coefficient: half at -N/2, half at +N/2
                const C<R> h0 = cscale(twisted(n), (R)0.5), h1 = cscale(twisted(-n), (R)0.5);
                lds[M + n] = h0;         // -N/2 mod M
                lds[-n] = h1;            // +N/2
            } else {
                lds[n < 0 ? M + n : n] = twisted(n);
            }
        }
    }
    __syncthreads();

    // 3) g = conj(DFT_M(conj(d))) on all T threads, stored in natural order
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = cconj(lds[t + T * e]);
    fft_lds<E>(v, lds, t, T, a.sc2);
#pragma unroll
    for (int e = 0; e < E; ++e)
        stc<R>(dst + t + T * e, cconj(v[e]));
}

// out[s][j] = fine[s][j + off], j < N (the fine transform's rows at y_j).
template <typename R>
__global__ void k_window(const typename Vec<R>::T *__restrict__ fine, typename Vec<R>::T *__restrict__ out, int N,
                         int M, int off, int64_t total)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / N;
        const int j = (int)(i - s * N);
        out[i] = fine[s * M + off + j];
    }
}

} // namespace lctk
