// cx_impl.hpp - the LCT of §1 for a complex matrix (a, b, d) evaluated by the
// Algorithm as printed, with complex parameters: the cross term
// -x_k y_j / b = -4 x_k x_j / pi does not depend on b, so the DFT and its index
// phases are those of the real case, and only the diagonals change:
//   pre  e^{i a x_k^2 / (2b)}    = exp(w_a x_k^2),  w_a = i a / (2b)
//   post e^{i d y_j^2 / (2b)}    = exp(w_d x_j^2),  w_d = 8 i b d / pi^2   (y_j = 4 b x_j / pi)
//   amp  h (2 pi i b)^(-1/2) e^{-i pi (N-1)^2 / (2N)}
// Gaussian-chirp diagonals (modulus <= 1 when Im(a/b) >= 0 and Im(bd) >= 0).
// The outputs sit at the complex nodes y_j = 4 b x_j / pi; (0, i, 0) is the
// bilateral Laplace transform on the imaginary axis.
#pragma once
#include "kernels_impl.hpp"

namespace lctk {

// The diagonal exp(w n^2) (n = 2p - N + 1) times the index phase
// (N - 1) p / (2N) at this thread's positions p = t + T e, e = 0, 1, ...
__device__ __forceinline__ GaussPoly cx_poly(double mag, double hi, double lo, int t, int T, int N, double inv2N)
{
    GaussPoly g = gauss_poly(mag, hi, lo, 2 * t - N + 1, 2 * T);
    g.ph.A = frac_turns(g.ph.A + index_turns(t, N, inv2N));
    g.ph.B = frac_turns(g.ph.B + index_turns(T, N, inv2N));
    return g;
}

template <typename R> struct CxDiag;
template <> struct CxDiag<float> {
    GaussPoly g;
    __device__ CxDiag(double mag, double hi, double lo, int t, int T, int N, double inv2N)
        : g(cx_poly(mag, hi, lo, t, T, N, inv2N))
    {
    }
    __device__ __forceinline__ C<float> at(int e) { return gauss_at(g, e); }
    // the phase alone (a diagonal of zero log-modulus rate)
    __device__ __forceinline__ C<float> phase(int e) { return chirp_at<float>(g.ph, e); }
};
template <> struct CxDiag<double> {
    // values in order e = 0, 1, ... (at(e) once per e): the phase walked by
    // products as ChirpSeq<double> (the library sine/cosine costs tens of FP64
    // operations per call), the modulus exp(mag m^2) from the exact m^2
    GaussPoly g;
    ChirpSeq<double> c;
    __device__ CxDiag(double mag, double hi, double lo, int t, int T, int N, double inv2N)
        : g(cx_poly(mag, hi, lo, t, T, N, inv2N)), c(g.ph)
    {
    }
    __device__ __forceinline__ C<double> at(int e) { return cscale(c.next(), exp(fmax(gauss_logmod(g, e), -1000.0))); }
    __device__ __forceinline__ C<double> phase(int) { return c.next(); }
};

// NFIX > 0: the length's compile-time radix schedule (E = 16); with
// NFIX / E >= 256 threads one signal per work-group.  HX: LDS exchanged in
// real and imaginary halves (lds_elems(N) R per signal).
template <typename R, int E, int NFIX = 0, int LB = max_block(sizeof(R) == 8, E), bool HX = false>
__global__ __launch_bounds__(LB, HX ? 3 : 1) void k_lct_cx(const typename Vec<R>::T *__restrict__ in,
                                                           typename Vec<R>::T *__restrict__ out, CxArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = NFIX > 0 ? NFIX : a.N;
    const int T = NFIX > 0 ? NFIX / E : a.T;
    constexpr bool ONE = NFIX > 0 && NFIX / E >= 256;
    const int sl = ONE ? 0 : (int)threadIdx.x / T;
    const int t = (int)threadIdx.x - sl * T;
    const int64_t sig = (int64_t)blockIdx.x * a.S + sl;
    const bool live = sig < a.batch;
    const double inv2N = 0.5 / (double)N;
    using V = typename Vec<R>::T;
    [[maybe_unused]] const V *src = in + (size_t)(live ? sig : 0) * N;
    [[maybe_unused]] V *dst = out + (size_t)(live ? sig : 0) * N;
    // FP32: one buffer descriptor per work-group over its live signals, the
    // element offsets constant (slots past the batch read zeros); FP64 keeps
    // plain loads and stores (its 128-bit buffer stores timed slower here)
    const int64_t first = (int64_t)blockIdx.x * a.S;
    const int64_t nlive = a.batch - first < a.S ? a.batch - first : a.S;
    [[maybe_unused]] const __amdgpu_buffer_rsrc_t rin =
        make_rsrc(in + first * N, (uint32_t)(nlive * N * (int64_t)sizeof(V)));
    [[maybe_unused]] const __amdgpu_buffer_rsrc_t rout =
        make_rsrc(out + first * N, (uint32_t)(nlive * N * (int64_t)sizeof(V)));
    [[maybe_unused]] const int voff = (sl * N + t) * (int)sizeof(V);
    [[maybe_unused]] const int sstep = T * (int)sizeof(V);
    C<R> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if constexpr (sizeof(R) == 4)
            v[e] = Buf<R>::load(rin, voff, e * sstep);
        else
            v[e] = live ? ldc<R>(src + t + T * e) : C<R>{(R)0, (R)0};
    }
    // A diagonal whose log-modulus rate is zero (Im(a/b) = 0 for the pre-,
    // Im(bd) = 0 for the post-diagonal) is a pure phase: the exponential is
    // skipped (a branch uniform over the launch).
    {
        CxDiag<R> pre(a.k.pre_mag, a.k.pre_hi, a.k.pre_lo, t, T, N, inv2N);
        if (a.k.pre_mag == 0.0) {
#pragma unroll
            for (int e = 0; e < E; ++e)
                v[e] = cmul(v[e], pre.phase(e));
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e)
                v[e] = cmul(v[e], pre.at(e));
        }
    }
    if constexpr (NFIX > 0 && HX)
        fft_lds_fixed_half<E, NFIX>(v, reinterpret_cast<R *>(smem_raw) + (size_t)sl * lds_elems(N), t);
    else if constexpr (NFIX > 0)
        fft_lds_fixed<E, NFIX>(v, smem + (size_t)sl * lds_elems(N), t);
    else
        fft_lds<E>(v, smem + (size_t)sl * lds_elems(N), t, T, a.sc);
    if (live) {
        CxDiag<R> post(a.k.post_mag, a.k.post_hi, a.k.post_lo, t, T, N, inv2N);
        const C<R> amp{(R)a.k.amp_re, (R)a.k.amp_im};
        auto store = [&](int e, C<R> y) {
            if constexpr (sizeof(R) == 4)
                Buf<R>::store(y, rout, voff, e * sstep);
            else
                stc<R>(dst + t + T * e, y);
        };
        if (a.k.post_mag == 0.0) {
#pragma unroll
            for (int e = 0; e < E; ++e)
                store(e, cmul(cmul(v[e], post.phase(e)), amp));
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e)
                store(e, cmul(cmul(v[e], post.at(e)), amp));
        }
    }
}

} // namespace lctk
