// frft_large_impl.hpp - the same-grid fractional transform when its length
// L = 2N convolution does not fit one work-group's LDS.
//
// g = C D IDFT(DFT(v) . DFT(t)) restricted to the first N outputs, with
// v = D f zero-padded (reversed for the Hankel form) and t the Gaussian-chirp
// Toeplitz kernel.  The length-L DFTs are four-step FFTs (L = L1 L2); the
// workspace holds two length-L regions per signal (R0 for v, R1 for t).
// Launches: [pass 1: column DFTs of v and t, twiddled, stored transposed]
// [pass 2: row DFTs of both, their product and the inverse transform's row
// step, in place in R0] [pass 3: the inverse's column DFTs -> out].  With one
// order for the whole batch, t is transformed once: pass 1 runs its columns
// for slot 0 only, a pass-2 launch finishes that spectrum in place in slot 0's
// R1 (SPEC_WRITE), and the per-signal pass 2 reads it there (SPEC_READ).
#pragma once
#include "fourstep_impl.hpp"

namespace lctk {

enum FrKind { FR_DATA = 0, FR_KERN = 1 };

template <typename R>
__device__ __forceinline__ FrConst fr_const_of(const FrLArgs &a, int64_t s)
{
    return a.Z2 != nullptr ? fr_const(a.N, a.Z2[2 * s], a.Z2[2 * s + 1], sizeof(R) == 8) : a.k;
}

// Pass 1 over columns n2 of the length-L sequence (element i = n1 L2 + n2).
// blockIdx.x < batch * tiles handles the data (FR_DATA), the rest the
// kernel sequence (FR_KERN).  NF > 0: the column length L1 = NF with its
// compile-time radix schedule.
// With E even, L1 = T1 E is even and i < N = L1 L2 / 2 exactly when
// n1 < L1 / 2, i.e. e < E / 2: the data's upper half is the zero padding, and
// the kernel is at m = i for e < E / 2 and at m = L - i from there on (both
// give m = N at i = N), so each value is formed once.
template <typename R, int E, int LB = max_block(sizeof(R) == 8, E), int NF = 0>
__global__ __launch_bounds__(LB) void k_frl1(
    const typename Vec<R>::T *__restrict__ in, typename Vec<R>::T *__restrict__ ws, FrLArgs a)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = a.N, L = a.L, L1 = a.L1, L2 = a.L2, Cc = a.C, T1 = a.T1;
    const int tiles = L2 / Cc;
    int64_t b = blockIdx.x;
    int kind = FR_DATA;
    if (b >= a.batch * tiles) {
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
    V *R0 = ws + (size_t)s * 2 * L;
    V *R1 = R0 + L;

    // element i = (t + T1 e) L2 + n2
    C<R> v[E];
    const int i0 = t * L2 + n2, Di = T1 * L2;
    if (kind == FR_DATA) {
        // e^{-P x_i^2} f_i, n_i = 2i - N + 1, zero beyond N
        GaussSeq<R> dch(k.dmag, k.dph_hi, k.dph_lo, 2 * i0 - N + 1, 2 * Di);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = i0 + Di * e;
            C<R> x = {(R)0, (R)0};
            if constexpr (E % 2 == 0) {
                if (e < E / 2) {
                    const C<R> w = dch.next();
                    if (!k.special)
                        x = cmul(ldc<R>(in + (size_t)s * N + (k.hankel ? N - 1 - i : i)), w);
                }
            } else {
                const C<R> w = dch.next();
                if (i < N && !k.special)
                    x = cmul(ldc<R>(in + (size_t)s * N + (k.hankel ? N - 1 - i : i)), w);
            }
            v[e] = x;
        }
    } else if constexpr (E % 2 == 0) {
        // kernel at m = i (e < E/2), m = L - i = (L - i0 - Di E/2) - Di (e - E/2) after
        GaussSeq<R> lo(k.kmag, k.kph_hi, k.kph_lo, i0, Di);
        GaussSeq<R> hi(k.kmag, k.kph_hi, k.kph_lo, L - i0 - Di * (E / 2), -Di);
#pragma unroll
        for (int e = 0; e < E; ++e)
            v[e] = e < E / 2 ? lo.next() : hi.next();
    } else {
        // kernel at m = i for i <= N, m = L - i = (L - i0) - Di e beyond
        GaussSeq<R> lo(k.kmag, k.kph_hi, k.kph_lo, i0, Di), hi(k.kmag, k.kph_hi, k.kph_lo, L - i0, -Di);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const C<R> a = lo.next(), b = hi.next();
            v[e] = i0 + Di * e <= N ? a : b;
        }
    }

    C<R> *lds = smem + (size_t)sl * lds_elems(L1);
    fft_any<R, E, NF>(v, lds, t, T1, a.sc1);

    {
        const double A = -(double)umod24(n2 * t, L) / (double)L;
        const double B = -(double)umod24(n2 * T1, L) / (double)L;
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
    V *dst = kind == FR_DATA ? R0 : R1;
#pragma unroll
    for (int e = 0; e < E; ++e)
        stc<R>(dst + (size_t)(n20 + sl2) * L1 + t2 + T1 * e, l2[lds_pad(t2 + T1 * e)]);
}

// Pass 2 over rows k1 (element n2 of row k1 at n2 L1 + k1): the length-L2
// DFTs of both regions finish the spectra V and K at k = k1 + L1 k2; the
// inverse transform of P = V K then starts in LDS.  With n = n2 + L2 n1,
//   sum_k P_k W_L^(-n k) = sum_k1 W_L1^(-n1 k1) [W_L^(-n2 k1) sum_k2 W_L2^(-n2 k2) P_(k1 + L1 k2)],
// and the conjugate of the bracket (the forward length-L2 DFT of conj(P),
// times W_L^(+n2 k1), W_L = e^(-2 pi i / L)) is stored into R0 at n2 L1 + k1.
// NF > 0: the row length L2 = NF with its compile-time radix schedule.
template <typename R, int E, int LB = max_block(sizeof(R) == 8, E), int NF = 0>
__global__ __launch_bounds__(LB) void k_frl2(typename Vec<R>::T *__restrict__ ws, FrLArgs a)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int L = a.L, L1 = a.L1, RR = a.RR, T2 = a.T2;
    const int tiles = L1 / RR;
    const int64_t b = blockIdx.x;
    const int64_t s = b / tiles;
    const int k10 = (int)(b - s * tiles) * RR;
    const int tid = (int)threadIdx.x;
    const int r = tid % RR;
    const int t = tid / RR;
    const int k1 = k10 + r;
    const bool write_spec = a.spec_mode == SPEC_WRITE; // launched over slot 0's rows only
    V *R0 = ws + (size_t)s * 2 * L;
    V *R1 = a.spec_mode == SPEC_NONE ? R0 + L : ws + L;

    C<R> v[E], w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const size_t i = (size_t)(t + T2 * e) * L1 + k1;
        if (!write_spec)
            v[e] = ldc<R>(R0 + i);
        w[e] = ldc<R>(R1 + i);
    }
    C<R> *lds = smem + (size_t)r * lds_elems(a.L2);
    if (a.spec_mode != SPEC_READ)
        fft_any<R, E, NF>(w, lds, t, T2, a.sc2);
    if (write_spec) {
#pragma unroll
        for (int e = 0; e < E; ++e)
            stc<R>(R1 + (size_t)(t + T2 * e) * L1 + k1, w[e]);
        return;
    }
    fft_any<R, E, NF>(v, lds, t, T2, a.sc2);
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = cconj(cmul(v[e], w[e]));
    fft_any<R, E, NF>(v, lds, t, T2, a.sc2);
    const double A = -(double)umod24(k1 * t, L) / (double)L;
    const double B = -(double)umod24(k1 * T2, L) / (double)L;
#pragma unroll
    for (int e = 0; e < E; ++e)
        stc<R>(R0 + (size_t)(t + T2 * e) * L1 + k1, cmul(v[e], cis_turns_from<R>(frac_turns(fma(B, (double)e, A)))));
}

// Pass 3 over columns n2: the length-L1 DFT over k1 of the contiguous
// R0[n2 L1 + k1] gives the conjugate of the inverse transform at
// j = n2 + L2 n1; transposed through LDS (consecutive threads, consecutive j)
// it is conjugated, multiplied by the diagonal and the constant, and the
// first N outputs are stored.  NF > 0: the column length L1 = NF with its
// compile-time radix schedule.  With E even the kept outputs j < N are the
// positions n1 < L1 / 2, i.e. e < E / 2.
template <typename R, int E, int LB = max_block(sizeof(R) == 8, E), int NF = 0>
__global__ __launch_bounds__(LB) void k_frl3(const typename Vec<R>::T *__restrict__ ws,
                                                                       typename Vec<R>::T *__restrict__ out, FrLArgs a)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = a.N, L = a.L, L1 = a.L1, L2 = a.L2, Cc = a.C, T1 = a.T1;
    const int tiles = L2 / Cc;
    const int64_t b = blockIdx.x;
    const int64_t s = b / tiles;
    const int n20 = (int)(b - s * tiles) * Cc;
    const FrConst k = fr_const_of<R>(a, s);
    if (k.special)
        return; // whole work-group: k_fr_special writes this signal
    const int tid = (int)threadIdx.x;
    const int sl = tid / T1;
    const int t = tid - sl * T1;
    const V *R0 = ws + (size_t)s * 2 * L;

    C<R> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = ldc<R>(R0 + (size_t)(n20 + sl) * L1 + t + T1 * e);
    C<R> *lds = smem + (size_t)sl * lds_elems(L1);
    fft_any<R, E, NF>(v, lds, t, T1, a.sc1);
    constexpr int EK = E % 2 == 0 ? E / 2 : E; // values that can hold a kept output
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EK; ++e)
        lds[lds_pad(t + T1 * e)] = v[e];
    __syncthreads();
    const int sl2 = tid % Cc;
    const int t2 = tid / Cc;
    const C<R> *l2 = smem + (size_t)sl2 * lds_elems(L1);
    // output j = (n20 + sl2 + L2 t2) + L2 T1 e, the first N kept
    const int j0 = n20 + sl2 + L2 * t2;
    GaussSeq<R> och(k.omag, k.oph_hi, k.oph_lo, 2 * j0 - N + 1, 2 * L2 * T1);
#pragma unroll
    for (int e = 0; e < EK; ++e) {
        const int n1 = t2 + T1 * e;
        const int j = j0 + L2 * T1 * e;
        const C<R> w = och.next();
        if (j < N) {
            C<R> y = cmul(cconj(l2[lds_pad(n1)]), w);
            y = cmul(y, C<R>{(R)k.cre, (R)k.cim});
            stc<R>(out + (size_t)s * N + j, y);
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

// The default widths (E = 16; FP64 also 8) also have an instantiation bounded
// at 256 threads, used whenever the work-group fits it: with the 1024-thread
// bound the pass-2 kernel, which holds a data row and a kernel row per thread,
// is held to 128 registers and spills.  Those also have compile-time radix
// schedules for the sub-lengths 64 .. 4096.
template <typename R, int E> constexpr bool has_tight_frl() { return E == 16 || (sizeof(R) == 8 && E == 8); }
#define LCT_FRL_FIXED_LIST(X) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

// Column factors 3 2^k and 5 2^k of passes 1 and 3 at the widths the planner
// gives them (FP32 24 / 20, FP64 12 / 10), with compile-time schedules.
#define LCT_FRL_FIX3_24(X) X(192) X(384) X(768) X(1536) X(3072)
#define LCT_FRL_FIX5_20(X) X(160) X(320) X(640) X(1280) X(2560)
#define LCT_FRL_FIX3_12(X) X(96) X(192) X(384) X(768) X(1536)
#define LCT_FRL_FIX5_10(X) X(80) X(160) X(320) X(640) X(1280)
// (passes 1 and 3 take the same arguments: a source, a destination, FrLArgs)
template <typename R>
using FrlColsKernel = void (*)(const typename Vec<R>::T *, typename Vec<R>::T *, FrLArgs);
template <typename R, int E>
inline FrlColsKernel<R> frl_cols_fixed(int L1, const Sched &sc, bool pass3)
{
    constexpr int LB = max_block(sizeof(R) == 8, E);
    if (!is_fixed_sched(sc, L1, E))
        return nullptr;
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return pass3 ? k_frl3<R, E, LB, n> : k_frl1<R, E, LB, n>;
    if constexpr (sizeof(R) == 4 && E == 24) {
        switch (L1) { LCT_FRL_FIX3_24(X) default: break; }
    } else if constexpr (sizeof(R) == 4 && E == 20) {
        switch (L1) { LCT_FRL_FIX5_20(X) default: break; }
    } else if constexpr (sizeof(R) == 8 && E == 12) {
        switch (L1) { LCT_FRL_FIX3_12(X) default: break; }
    } else if constexpr (sizeof(R) == 8 && E == 10) {
        switch (L1) { LCT_FRL_FIX5_10(X) default: break; }
    }
#undef X
    return nullptr;
}

template <typename R, int E>
inline hipError_t launch_frl1_t(const void *in, void *ws, const FrLArgs &a, int nb, int bs, size_t lds, hipStream_t st)
{
    using V = typename Vec<R>::T;
    auto kern = k_frl1<R, E>;
    if constexpr (has_tight_frl<R, E>()) {
        if (bs <= 256) {
            kern = k_frl1<R, E, 256>;
            if (is_fixed_sched(a.sc1, a.L1, E)) {
                switch (a.L1) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        kern = k_frl1<R, E, 256, n>;                                                                                 \
        break;
                    LCT_FRL_FIXED_LIST(X)
#undef X
                default:
                    break;
                }
            }
        }
    }
    if constexpr (!has_tight_frl<R, E>()) {
        if (FrlColsKernel<R> f = frl_cols_fixed<R, E>(a.L1, a.sc1, false))
            kern = f;
    }
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, st, (const V *)in, (V *)ws, a);
    return hipGetLastError();
}

template <typename R, int E>
inline hipError_t launch_frl2_t(void *ws, const FrLArgs &a, int nb, int bs, size_t lds, hipStream_t st)
{
    using V = typename Vec<R>::T;
    auto kern = k_frl2<R, E>;
    if constexpr (has_tight_frl<R, E>()) {
        if (bs <= 256) {
            kern = k_frl2<R, E, 256>;
            if (is_fixed_sched(a.sc2, a.L2, E)) {
                switch (a.L2) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        kern = k_frl2<R, E, 256, n>;                                                                                 \
        break;
                    LCT_FRL_FIXED_LIST(X)
#undef X
                default:
                    break;
                }
            }
        }
    }
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, st, (V *)ws, a);
    return hipGetLastError();
}

template <typename R, int E>
inline hipError_t launch_frl3_t(const void *ws, void *out, const FrLArgs &a, int nb, int bs, size_t lds,
                                hipStream_t st)
{
    using V = typename Vec<R>::T;
    auto kern = k_frl3<R, E>;
    if constexpr (has_tight_frl<R, E>()) {
        if (bs <= 256) {
            kern = k_frl3<R, E, 256>;
            if (is_fixed_sched(a.sc1, a.L1, E)) {
                switch (a.L1) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        kern = k_frl3<R, E, 256, n>;                                                                                 \
        break;
                    LCT_FRL_FIXED_LIST(X)
#undef X
                default:
                    break;
                }
            }
        }
    }
    if constexpr (!has_tight_frl<R, E>()) {
        if (FrlColsKernel<R> f = frl_cols_fixed<R, E>(a.L1, a.sc1, true))
            kern = f;
    }
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, st, (const V *)ws, (V *)out, a);
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
