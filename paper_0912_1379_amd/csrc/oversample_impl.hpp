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

// Compile-time-schedule version (E = 16) of fft_lds_part.
template <int E, int N, int S, int NS, typename R>
__device__ __forceinline__ void fft_lds_part_fixed(C<R> *v, C<R> *lds, int t, bool active)
{
    constexpr int NST = fixed_nstages(N, E);
    if constexpr (S < NST) {
        constexpr int RAD = fixed_radix(N, E, S);
        constexpr int T = N / E;
        if (active)
            stage_compute<E, RAD>(v, t, T, NS);
        if constexpr (S + 1 < NST) {
            __syncthreads();
            if (active)
                stage_write<E, RAD>(lds, v, t, T, NS);
            __syncthreads();
            if (active)
                stage_read<E>(lds, v, t, T);
        }
        fft_lds_part_fixed<E, N, S + 1, NS * RAD>(v, lds, t, active);
    }
}

// One signal per work-group.  With c_n = (1/N) sum_k f_k e^{-2 pi i n k / N}
// (n = k for k < N/2, k - N above; for even N the coefficient at n = -N/2 is
// split in halves between -N/2 and +N/2), the fine samples are
//   g_m = sum_n c_n e^{-i pi n (P - 1) / (P N)} e^{2 pi i n m / (P N)},
// i.e. f's trigonometric interpolant at x_0 + (h / P)(m - (P - 1)/2).
// NF1, NF2 > 0: the lengths N and P N with their compile-time schedules (E = 16).
template <typename R, int E, int NF1 = 0, int NF2 = 0>
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
    if constexpr (NF1 > 0)
        fft_lds_part_fixed<E, NF1, 0, 1>(v, lds, t, act);
    else
        fft_lds_part<E>(v, lds, t, T1, a.sc1, act);

    // 2) the zero-padded, twisted coefficients in natural order (LDS, unpadded)
    __syncthreads(); // the DFT's last exchange has been read
    for (int i = t; i < M; i += T)
        lds[i] = C<R>{(R)0, (R)0};
    __syncthreads();
    if (act) {
        const R inv = (R)1 / (R)N;
        const double inv2M = 0.5 / (double)M;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + T1 * e;
            const int n = k < (N + 1) / 2 ? k : k - N; // -floor(N/2) .. ceil(N/2) - 1
            const C<R> c = cscale(v[e], inv);
            // twist e^{-i pi n (P-1) / (P N)}: -n (P-1) / (2 M) turns; |n (P-1)| < M
            // (|n| <= N/2), so the integer product is exact and the turns lie in
            // (-1/2, 1/2) without a reduction
            auto twisted = [&](int nn) { return cmul(c, cis_turns_from<R>(-(double)(nn * (P - 1)) * inv2M)); };
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
    if constexpr (NF2 > 0)
        fft_lds_fixed<E, NF2>(v, lds, t);
    else
        fft_lds<E>(v, lds, t, T, a.sc2);
#pragma unroll
    for (int e = 0; e < E; ++e)
        stc<R>(dst + t + T * e, cconj(v[e]));
}

// The interpolation (as k_interp), the LCT of the P N fine samples (pre-chirp,
// DFT, post-chirp with the constants a.k) and the window [(P - 1) N / 2,
// (P + 1) N / 2) in one work-group per signal: the fine samples never leave
// LDS and registers.  Compile-time schedules for N and M = P N at E values
// per thread (T = M / E <= LB threads).  FP64 takes LB = 512 (256 VGPRs per
// thread): at 1024 threads the 128-register cap spills.
// With 2P dividing E, N / 2 is a whole number of thread strides T, so the
// zero-padded spectrum's support [0, N/2] and [M - N/2, M) is, in the layout
// t + T e, the values e < EL and e >= E - EL (EL = E / 2P) of every thread and
// e = EL of thread 0 (position N/2, the upper half of the Nyquist
// coefficient): the other values are zeros known at compile time, and the
// zero fill of LDS is not needed.  Likewise the window is the values
// e in [E0, E0 + N / T) (E0 = (P - 1) N / 2T) of every thread.
template <typename R, int E, int NF1, int NF2, int LB = 1024>
__global__ __launch_bounds__(LB) void k_os_fused(const typename Vec<R>::T *__restrict__ in,
                                                   typename Vec<R>::T *__restrict__ out, InterpArgs a)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *lds = reinterpret_cast<C<R> *>(smem_raw);
    constexpr int N = NF1, M = NF2, T = M / E, T1 = N / E, P = M / N;
    static_assert(M % N == 0 && P >= 2 && N % 2 == 0 && E % (2 * P) == 0, "spectrum support in whole strides");
    constexpr int EL = E / (2 * P);
    constexpr int OFF = (P - 1) * N / 2, E0 = OFF / T, NW = N / T;
    static_assert(OFF % T == 0 && N % T == 0 && E0 + NW <= E, "window in whole strides");
    const int t = (int)threadIdx.x;
    const int64_t s = blockIdx.x;
    const bool act = t < T1;
    const V *src = in + (size_t)s * N;

    // 1) c = DFT_N(f) / N on the first T1 threads
    C<R> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = act ? ldc<R>(src + t + T1 * e) : C<R>{(R)0, (R)0};
    fft_lds_part_fixed<E, N, 0, 1>(v, lds, t, act);

    // 2) the twisted coefficients at their positions of the length-M spectrum
    //    (natural order, unpadded; only the support is written)
    __syncthreads(); // the DFT's last exchange has been read
    if (act) {
        const R inv = (R)1 / (R)N;
        const double inv2M = 0.5 / (double)M;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + T1 * e;
            const int n = k < N / 2 ? k : k - N; // -N/2 .. N/2 - 1
            const C<R> c = cscale(v[e], inv);
            auto twisted = [&](int nn) { return cmul(c, cis_turns_from<R>(-(double)(nn * (P - 1)) * inv2M)); };
            if (2 * n == -N) {
                const C<R> h0 = cscale(twisted(n), (R)0.5), h1 = cscale(twisted(-n), (R)0.5);
                lds[M + n] = h0;
                lds[-n] = h1;
            } else {
                lds[n < 0 ? M + n : n] = twisted(n);
            }
        }
    }
    __syncthreads();

    // 3) the fine samples g = conj(DFT_M(conj(d))), kept in registers
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e < EL || e >= E - EL)
            v[e] = cconj(lds[t + T * e]);
        else if (e == EL)
            v[e] = t == 0 ? cconj(lds[T * EL]) : C<R>{(R)0, (R)0};
        else
            v[e] = C<R>{(R)0, (R)0};
    }
    fft_lds_fixed<E, M>(v, lds, t);

    // 4) the fine-grid LCT: pre-chirp, DFT, post-chirp; the window stored
    const LctConst &k = a.k;
    const double inv2M = 0.5 / (double)M;
    {
        ChirpSeq<R> cin(thread_chirp(k.pre_hi, k.pre_lo, true, t, T, M, inv2M));
#pragma unroll
        for (int e = 0; e < E; ++e)
            v[e] = cmul(cconj(v[e]), cin.next());
    }
    fft_lds_fixed<E, M>(v, lds, t);
    {
        const R mag = (R)k.amp_mag;
        ChirpSeq<R> cout(seq_chirp(k.post_hi, k.post_lo, true, t + OFF, T, M, inv2M, k.amp_turns));
        V *dst = out + (size_t)s * N;
#pragma unroll
        for (int e = 0; e < NW; ++e)
            stc<R>(dst + t + T * e, cscale(cmul(v[E0 + e], cout.next()), mag));
    }
}

// out[s][j] = fine[s][j + off], j < N (the fine transform's rows at y_j).
// Grid: (ceil(N / blockDim), up to 65535 signal rows, each row striding over
// the batch); no division per element.
template <typename R>
__global__ void k_window(const typename Vec<R>::T *__restrict__ fine, typename Vec<R>::T *__restrict__ out, int N,
                         int M, int off, int64_t batch)
{
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= N)
        return;
    for (int64_t s = blockIdx.y; s < batch; s += gridDim.y)
        out[s * N + j] = fine[s * M + off + j];
}

} // namespace lctk
