// kernels_impl.hpp - single-pass (in-LDS) kernels of the discrete LCT and of
// the same-grid fractional transform for gfx950.
//
// One work-group holds S signals of N points; each signal is processed by
// T = N / E threads that own E complex values each (see fft_core.hpp).  The
// chirp-scaling diagonals of the Algorithm (steps 1 and 2) are applied while
// the samples travel between HBM and registers, so HBM sees exactly one read
// and one write per sample.
#pragma once
#include "lct_kernels.hpp"

#include "fft_core.hpp"
#include "lct_params.hpp"
#include "mfma_fft.hpp"

namespace lctk {

enum Mode { MODE_FWD = 0, MODE_ADJ = 1 };

// n^2 for n = 2i - N + 1, exact in double for N < 2^26.
__device__ __forceinline__ double nsq(int i, int N)
{
    double n = (double)(2 * i - N + 1);
    return n * n;
}

template <typename R>
__device__ __forceinline__ C<R> pre_factor(const LctConst &k, int i, int N, double inv2N)
{
    double t = quad_turns(Quad{k.pre_hi, k.pre_lo}, nsq(i, N)) + index_turns(i, N, inv2N);
    return cis_turns_from<R>(frac_turns(t));
}

template <typename R>
__device__ __forceinline__ C<R> post_factor(const LctConst &k, int j, int N, double inv2N)
{
    double t = quad_turns(Quad{k.post_hi, k.post_lo}, nsq(j, N)) + index_turns(j, N, inv2N);
    C<R> c = cis_turns_from<R>(frac_turns(t));
    return cmul(c, C<R>{(R)k.amp_re, (R)k.amp_im});
}

// Quadratic phase of the positions i_e = t + T e a thread owns, as a
// polynomial in e:  q n_e^2 (+ (N-1) i_e / (2N))  =  A + e B + e^2 C  (turns),
// n_e = n_t + 2 T e.  A, B, C are reduced modulo 1 once per thread from exact
// integers, so each element costs two FMAs and one reduction.
struct ThreadChirp {
    double A, B, C;
};

__device__ __forceinline__ ThreadChirp thread_chirp(double qhi, double qlo, bool with_index, int t, int T, int N,
                                                    double inv2N, double extra_turns = 0.0)
{
    const Quad q{qhi, qlo};
    const double nt = (double)(2 * t - N + 1);
    double A = quad_turns(q, nt * nt) + extra_turns;
    double B = quad_turns(q, 4.0 * (double)T * nt);
    double C = quad_turns(q, 4.0 * (double)T * (double)T);
    if (with_index) {
        A += index_turns(t, N, inv2N);
        B += index_turns(T, N, inv2N);
    }
    return {frac_turns(A), frac_turns(B), frac_turns(C)};
}

// Same polynomial for the positions i_e = i0 + D e (any stride D):
// n_e = n_{i0} + 2 D e.  Needs |n| < 2^24 so that every product is exact.
__device__ __forceinline__ ThreadChirp seq_chirp(double qhi, double qlo, bool with_index, int i0, int D, int N,
                                                 double inv2N, double extra_turns = 0.0)
{
    const Quad q{qhi, qlo};
    const double n0 = (double)(2 * i0 - N + 1);
    double A = quad_turns(q, n0 * n0) + extra_turns;
    double B = quad_turns(q, 4.0 * (double)D * n0);
    double C = quad_turns(q, 4.0 * (double)D * (double)D);
    if (with_index) {
        A += index_turns(i0, N, inv2N);
        B += index_turns(D, N, inv2N);
    }
    return {frac_turns(A), frac_turns(B), frac_turns(C)};
}

template <typename R>
__device__ __forceinline__ C<R> chirp_at(const ThreadChirp &c, int e)
{
    const double fe = (double)e;
    double u = fma(c.B, fe, fma(c.C, fe * fe, c.A));
    return cis_turns_from<R>(frac_turns(u));
}

// The chirp values c_e = cis(A + e B + e^2 C) of one thread, e = 0, 1, 2, ...
// in order (next() once per e).  FP32: each from its phase (hardware
// sine/cosine).  FP64: the library sine/cosine costs tens of FP64 operations
// per call, so the sequence is walked by products instead,
//   c_{e+1} = c_e d_e,  d_e = cis(B + (2e + 1) C),  d_{e+1} = d_e cis(2 C),
// from three evaluations per thread; after e steps the error is about 2 e^2
// rounding units (4e-14 at e = 15), half that of summing the phase polynomial
// in FP64 for each value, whose rounding grows with e^2 |C| turns.
template <typename R> struct ChirpSeq;
template <> struct ChirpSeq<float> {
    ThreadChirp p;
    int e;
    __device__ explicit ChirpSeq(const ThreadChirp &c) : p(c), e(0) {}
    __device__ __forceinline__ C<float> next() { return chirp_at<float>(p, e++); }
};
template <> struct ChirpSeq<double> {
    C<double> c, d, r;
    __device__ explicit ChirpSeq(const ThreadChirp &p)
        : c(cis_turns(p.A)), d(cis_turns(frac_turns(p.B + p.C))), r(cis_turns(frac_turns(2.0 * p.C)))
    {
    }
    __device__ __forceinline__ C<double> next()
    {
        const C<double> o = c;
        c = cmul(c, d);
        d = cmul(d, r);
        return o;
    }
};

// ---------------------------------------------------------------------------
// LCT forward (MODE_FWD) / adjoint (MODE_ADJ).  Per-signal constants come from
// args.k (one matrix for the batch) or are derived from M4[sig].
//   forward: load f, times pre-chirp; DFT; times post-chirp and amplitude.
//   adjoint: L^H g = conj(pre (DFT(post conj(g)))) (the DFT matrix is symmetric).
// ---------------------------------------------------------------------------
// MF: radix-16 stages on the matrix cores (FP32 data, E = 16, split-BF16
// products; see mfma_fft.hpp).  HX (fixed lengths): LDS exchanges in real and
// imaginary halves, lds_elems(N) R of LDS per signal, and at least three waves
// per SIMD asked of the register allocation.
// WIN (forward, fixed lengths): only the outputs at positions
// [win_off, win_off + win_n) are stored, as win_n contiguous values per signal.
template <typename R, int E, int NFIX, int MODE, bool MF = false, int LB = max_block(sizeof(R) == 8, E),
          bool HX = false, bool WIN = false>
__global__ __launch_bounds__(LB, HX ? 3 : 1) void k_lct(
    const typename Vec<R>::T *__restrict__ in, typename Vec<R>::T *__restrict__ out, LctArgs args)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);

    const int N = NFIX > 0 ? NFIX : args.N;
    const int T = NFIX > 0 ? NFIX / E : args.T;

    // The fixed-size instantiation is launched with one signal per
    // work-group (T = NFIX / E >= 256 threads); saying so at compile time
    // keeps the signal index uniform (scalar loads of its parameters).
    constexpr bool ONE = NFIX > 0 && NFIX / E >= 256;
    const int sl = ONE ? 0 : (int)threadIdx.x / T; // signal slot within the work-group
    const int t = (int)threadIdx.x - sl * T;
    const int64_t sig = (int64_t)blockIdx.x * args.S + sl;
    const bool live = sig < args.batch;
    C<R> *lds = smem + (size_t)sl * lds_elems(N);
    const double inv2N = 0.5 / (double)N;

    // Per-signal matrix, loaded before the samples so that waiting for it
    // does not wait for them.
    double m4[4] = {0.0, 0.0, 0.0, 0.0};
    if (args.M4 != nullptr) {
        const int64_t ss = live ? sig : 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            m4[q] = args.M4[4 * ss + q];
    }

    // One buffer descriptor per work-group covering its live signals; thread
    // t of slot sl reads/writes element t + T e at voff + e * (T * sizeof(V)).
    const int64_t first = (int64_t)blockIdx.x * args.S;
    const int64_t nlive = args.batch - first < args.S ? args.batch - first : args.S;
    const uint32_t wg_bytes = (uint32_t)(nlive * N * (int64_t)sizeof(V));
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(in + first * N, wg_bytes);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(out + first * N, wg_bytes);
    const int voff = (sl * N + t) * (int)sizeof(V);
    const int sstep = T * (int)sizeof(V);

    // Issue every load first: the per-signal constants below are computed
    // while the samples are in flight.
    C<R> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = Buf<R>::load(rin, voff, e * sstep);

    const LctConst k = args.M4 != nullptr ? lct_const_from(args.nc, m4[0], m4[1], m4[2], m4[3]) : args.k;
    const R mag = (R)k.amp_mag;

    if (k.b0) {
        // b = 0 (§1): a diagonal, no DFT.  Write it now and join the FFT
        // with zeros so the work-group's barriers stay uniform.
        ChirpSeq<R> cb(thread_chirp(k.post_hi, k.post_lo, false, t, T, N, inv2N, k.amp_turns));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            C<R> f = cscale(cb.next(), mag);
            Buf<R>::store(cmul(v[e], MODE == MODE_FWD ? f : cconj(f)), rout, voff, e * sstep);
            v[e] = C<R>{(R)0, (R)0};
        }
    } else {
        ChirpSeq<R> cin(MODE == MODE_FWD ? thread_chirp(k.pre_hi, k.pre_lo, true, t, T, N, inv2N)
                                         : thread_chirp(k.post_hi, k.post_lo, true, t, T, N, inv2N, k.amp_turns));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (MODE == MODE_FWD)
                v[e] = cmul(v[e], cin.next());
            else
                v[e] = cscale(cmul(cconj(v[e]), cin.next()), mag);
        }
    }

    if constexpr (MF) {
        static_assert(E == 16 && sizeof(R) == 4 && NFIX == 0, "matrix-core stages: FP32, E = 16");
        fft_lds_mfma(v, smem, sl, t, T, N, lds_elems(N), args.sc);
    } else if constexpr (NFIX > 0) {
        if constexpr (HX)
            fft_lds_fixed_half<E, NFIX>(v, reinterpret_cast<R *>(smem_raw) + (size_t)sl * lds_elems(N), t);
        else
            fft_lds_fixed<E, NFIX>(v, lds, t);
    } else {
        fft_lds<E>(v, lds, t, T, args.sc);
    }

    if (live && !k.b0) {
        ChirpSeq<R> cout(MODE == MODE_FWD ? thread_chirp(k.post_hi, k.post_lo, true, t, T, N, inv2N, k.amp_turns)
                                          : thread_chirp(k.pre_hi, k.pre_lo, true, t, T, N, inv2N));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            C<R> y;
            if constexpr (MODE == MODE_FWD)
                y = cscale(cmul(v[e], cout.next()), mag);
            else
                y = cconj(cmul(v[e], cout.next()));
            if constexpr (WIN) {
                const unsigned q = (unsigned)(t + T * e - args.win_off);
                if (q < (unsigned)args.win_n)
                    stc<R>(out + sig * args.win_n + q, y);
            } else {
                Buf<R>::store(y, rout, voff, e * sstep);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Parameter gradient.  b != 0: G = L f and H = L(i x_k^2/(2b) f) in LDS, then
// per-signal sums  S_H = Re sum conj(g) H,  S_G = Re sum conj(g) G,
// S_n = Re sum conj(g) i (n_j^2 / N) G, combined into
// dl/da = S_H, dl/db = -S_G/(2b) - (a/b) S_H + d S_n, dl/dc = 0, dl/dd = b S_n.
// b = 0 (the diagonal of §1, G_j = sqrt(d) e^{i c x_j^2/(2d)} f_j, output
// nodes x_j/d): dG_j/dc = i x_j^2/(2d) G_j and dG_j/dd = (1/(2d) - i c x_j^2/(2d^2)) G_j,
// so with x_j^2 = pi^2 n_j^2/(8N) the same S_G and S_n give
// dl/dc = pi^2 S_n / (16 d), dl/dd = S_G/(2d) - (c/d) dl/dc, dl/da = dl/db = 0.
// Such a signal joins the work-group's FFTs (their barriers are uniform) and
// ignores their results.
// The sums are reduced in a fixed order (a tree over the slot's threads in
// LDS), so the gradient is the same bit for bit on every run.
// ---------------------------------------------------------------------------
// Sum of one value per thread of a signal slot (T threads, buf holds at least T
// doubles of the slot's own LDS); every thread of the work-group calls it.
__device__ __forceinline__ double slot_sum(double v, double *buf, int t, int T)
{
    __syncthreads();
    buf[t] = v;
    __syncthreads();
    int w = 1;
    while (w < T)
        w <<= 1;
    for (w >>= 1; w >= 1; w >>= 1) {
        if (t < w && t + w < T)
            buf[t] += buf[t + w];
        __syncthreads();
    }
    return buf[0];
}

template <typename R, int E, int NFIX = 0, int LB = max_block(sizeof(R) == 8, E)>
__global__ __launch_bounds__(LB) void k_lct_pgrad(
    const typename Vec<R>::T *__restrict__ f, const typename Vec<R>::T *__restrict__ g,
    double *__restrict__ grad4, LctArgs args)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = NFIX > 0 ? NFIX : args.N;
    const int T = NFIX > 0 ? NFIX / E : args.T;
    const Sched &sc = args.sc;
    const int sl = (int)threadIdx.x / T;
    const int t = (int)threadIdx.x - sl * T;
    const int64_t sig = (int64_t)blockIdx.x * args.S + sl;
    const bool live = sig < args.batch;
    C<R> *lds = smem + (size_t)sl * lds_elems(N);
    const double inv2N = 0.5 / (double)N;
    const int64_t ss = live ? sig : 0;
    const double a = args.M4[4 * ss + 0], b = args.M4[4 * ss + 1], c = args.M4[4 * ss + 2],
                 d = args.M4[4 * ss + 3];
    const LctConst k = lct_const_from(args.nc, a, b, c, d);
    const V *fs = f + (size_t)ss * N;
    const V *gs = g + (size_t)ss * N;

    // x_k^2 / (2b) = pi^2 n_k^2 / (16 b N)
    const double qscale = k.b0 ? 0.0 : PI_HI * PI_HI / (16.0 * b * (double)N);
    double sH = 0.0, sG = 0.0, sN = 0.0;
    C<R> v[E];
    for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = t + T * e;
            C<R> x = live && !k.b0 ? ldc<R>(fs + i) : C<R>{(R)0, (R)0};
            x = cmul(x, pre_factor<R>(k, i, N, inv2N));
            if (pass == 0)
                x = cmul_pi(cscale(x, (R)(qscale * nsq(i, N))));
            v[e] = x;
        }
        if constexpr (NFIX > 0)
            fft_lds_fixed<E, NFIX>(v, lds, t);
        else
            fft_lds<E>(v, lds, t, T, sc);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = t + T * e;
            if (!live || (k.b0 && pass == 0))
                continue;
            C<R> y;
            if (k.b0) {
                // the diagonal: sqrt(d) e^{i c x_j^2/(2d)} f_j
                const double tj = quad_turns(Quad{k.post_hi, k.post_lo}, nsq(j, N)) + k.amp_turns;
                y = cmul(ldc<R>(fs + j), cscale(cis_turns_from<R>(frac_turns(tj)), (R)k.amp_mag));
            } else {
                y = cmul(v[e], post_factor<R>(k, j, N, inv2N));
            }
            C<R> gj = ldc<R>(gs + j);
            // Re(conj(g) y)
            double re = (double)gj.x * (double)y.x + (double)gj.y * (double)y.y;
            if (pass == 0) {
                sH += re;
            } else {
                sG += re;
                // Re(conj(g) i y) = gj.x * (-y.y) + gj.y * y.x
                double im = -(double)gj.x * (double)y.y + (double)gj.y * (double)y.x;
                sN += im * nsq(j, N) / (double)N;
            }
        }
    }
    // the slot's FFT area (at least N complex values) holds the T partial sums
    double *buf = reinterpret_cast<double *>(lds);
    const double SH = slot_sum(sH, buf, t, T);
    const double SG = slot_sum(sG, buf, t, T);
    const double SN = slot_sum(sN, buf, t, T);
    if (live && t == 0) {
        if (k.b0) {
            const double gc = PI_HI * PI_HI * SN / (16.0 * d);
            grad4[4 * sig + 0] = 0.0;
            grad4[4 * sig + 1] = 0.0;
            grad4[4 * sig + 2] = gc;
            grad4[4 * sig + 3] = SG / (2.0 * d) - (c / d) * gc;
        } else {
            grad4[4 * sig + 0] = SH;
            grad4[4 * sig + 1] = -SG / (2.0 * b) - (a / b) * SH + d * SN;
            grad4[4 * sig + 2] = 0.0;
            grad4[4 * sig + 3] = b * SN;
        }
    }
}

// ---------------------------------------------------------------------------
// Same-grid fractional transform: length-L (L = 2N) FFT convolution
//   g_j = C e^{-P x_j^2} sum_k T_{j-k} e^{-P x_k^2} f_k (Toeplitz) or with the
// input reversed (Hankel).  Three FFTs in LDS: the kernel's spectrum (kept in
// registers at the positions each thread owns after an FFT), the data's
// spectrum, and the inverse of their product (as conj(FFT(conj(.)))).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ C<R> gauss_chirp(double mag_per, double ph_hi, double ph_lo, double m2)
{
    double lm = mag_per * m2;              // log modulus (<= 0)
    double t = quad_turns(Quad{ph_hi, ph_lo}, m2);
    C<R> c = cis_turns_from<R>(frac_turns(t));
    R s;
    if constexpr (sizeof(R) == 4)
        s = expf((float)fmax(lm, -200.0));
    else
        s = exp(fmax(lm, -1000.0));
    return cscale(c, s);
}

// The Gaussian-chirp values exp(mag m^2) cis(ph m^2) of one thread at
// m_e = m0 + D e, e = 0, 1, 2, ... in order (next() once per e).  The turns
// ph m_e^2 are the quadratic A + e B + e^2 C whose coefficients are formed
// once per thread from the exact integers m0^2, 2 m0 D and D^2 and reduced
// modulo 1 in double-double (as quad_turns does for m^2 itself), so a value
// costs two FP64 fused multiply-adds and one reduction instead of a
// double-double product.  The log-modulus mag m_e^2 is formed from the exact
// m_e^2 (a quadratic in e would cancel large terms where m0 is large and m_e
// small).  FP32 evaluates the phase with the hardware sine/cosine; FP64 walks
// it by products (as ChirpSeq<double>, about 2 e^2 rounding units after e
// steps).
struct GaussPoly {
    double mag;
    int m0, D;
    ThreadChirp ph; // turns
};
__device__ __forceinline__ GaussPoly gauss_poly(double mag_per, double ph_hi, double ph_lo, int m0, int D)
{
    const double a = (double)m0 * (double)m0, b = 2.0 * (double)m0 * (double)D, c = (double)D * (double)D;
    const Quad q{ph_hi, ph_lo};
    return {mag_per, m0, D, {frac_turns(quad_turns(q, a)), frac_turns(quad_turns(q, b)), frac_turns(quad_turns(q, c))}};
}
__device__ __forceinline__ double gauss_logmod(const GaussPoly &g, int e)
{
    const double m = (double)(g.m0 + g.D * e);
    return g.mag * (m * m);
}
// FP32: the value at any e (no state beyond the coefficients).  The modulus
// is 2^x by the hardware base-2 exponential, x = log2(e) mag m^2 formed in
// FP64 and rounded to FP32 once (the exponent's rounding is then that of the
// natural-log exponent rounded for expf; the library expf costs about ten
// more instructions per value).  x below the FP32 range gives 0.
__device__ __forceinline__ C<float> gauss_at(const GaussPoly &g, int e)
{
    const double m = (double)(g.m0 + g.D * e);
    const float x = (float)((g.mag * 1.4426950408889634074) * (m * m));
    return cscale(chirp_at<float>(g.ph, e), __builtin_amdgcn_exp2f(x));
}
template <typename R> struct GaussSeq;
template <> struct GaussSeq<float> {
    GaussPoly g;
    int e;
    __device__ GaussSeq(double mag_per, double ph_hi, double ph_lo, int m0, int D)
        : g(gauss_poly(mag_per, ph_hi, ph_lo, m0, D)), e(0)
    {
    }
    __device__ __forceinline__ C<float> next() { return gauss_at(g, e++); }
};
template <> struct GaussSeq<double> {
    GaussPoly g;
    ChirpSeq<double> c;
    int e;
    __device__ GaussSeq(double mag_per, double ph_hi, double ph_lo, int m0, int D)
        : g(gauss_poly(mag_per, ph_hi, ph_lo, m0, D)), c(g.ph), e(0)
    {
    }
    __device__ __forceinline__ C<double> next() { return cscale(c.next(), exp(fmax(gauss_logmod(g, e++), -1000.0))); }
};

// Launch bound of a fixed-length instantiation (E = 16): the work-group of the
// default geometry, max(256, length / 16) threads, so that the register
// budget is not cut to what 1024 threads would allow.
constexpr int tight_bound(int n) { return n / 16 > 256 ? n / 16 : 256; }

// The in-LDS FFT with a compile-time schedule when NF > 0, else the runtime
// one; DB: the double-buffered exchange (lds1 the second buffer, par the
// alternation state shared by the kernel's FFTs).
template <typename R, int E, int NF, bool DB = false>
__device__ __forceinline__ void fft_any(C<R> *v, C<R> *lds, int t, int T, const Sched &sc, C<R> *lds1 = nullptr,
                                        int *par = nullptr)
{
    if constexpr (DB)
        fft_lds_fixed2<E, NF>(v, lds, lds1, t, *par);
    else if constexpr (NF > 0)
        fft_lds_fixed<E, NF>(v, lds, t);
    else
        fft_lds<E>(v, lds, t, T, sc);
}

// LFIX > 0: the convolution length L = 2N = LFIX with its compile-time radix
// schedule.  SREAD: the instantiation for a spectrum shared by the batch
// (SPEC_READ), which reads it from the workspace at the product instead of
// holding it in registers through the data's FFT; with those registers free
// it is asked for four waves per SIMD (FP32: two 512-thread work-groups per CU
// at L = 8192, against one for the kernel that transforms its own spectrum),
// FP64 below 1024 threads for two (its LDS holds it to one work-group per CU
// at L = 8192; four waves would cut it to 128 registers and spill).
// DB (fixed lengths): the FFT exchanges alternate between two LDS buffers
// (twice the LDS, one barrier per stage); used where the registers already
// hold the work-group to one per CU.
template <typename R, int E, int LFIX = 0, int LB = max_block(sizeof(R) == 8, E), bool SREAD = false,
          bool DB = false>
__global__ __launch_bounds__(LB, SREAD ? (sizeof(R) == 8 && LB < 1024 ? 2 : 4) : 1) void k_frft(
    const typename Vec<R>::T *__restrict__ in, typename Vec<R>::T *__restrict__ out, FrArgs args)
{
    using V = typename Vec<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = LFIX > 0 ? LFIX / 2 : args.N;
    const int L = 2 * N;
    const int T = LFIX > 0 ? LFIX / E : args.T; // = L / E
    const Sched &sc = args.sc;
    const int sl = (int)threadIdx.x / T;
    const int t = (int)threadIdx.x - sl * T;
    const int64_t sig = (int64_t)blockIdx.x * args.S + sl;
    const bool live = sig < args.batch;
    C<R> *lds = smem + (size_t)sl * lds_elems(L);
    C<R> *lds1 = DB ? smem + (size_t)(args.S + sl) * lds_elems(L) : nullptr;
    int par = 0;
    const int64_t ss = live ? sig : 0;
    FrConst k = args.Z2 ? fr_const(N, args.Z2[2 * ss], args.Z2[2 * ss + 1], sizeof(R) == 8) : args.k;
    const V *src = in + (size_t)ss * N;
    V *dst = out + (size_t)ss * N;

    if (k.special) {
        // z = +-1: continuum limits (no FFT); keep the barrier pattern uniform
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int j = t + T * e; // < N
            if (live) {
                C<R> x = ldc<R>(src + (k.special == 1 ? j : N - 1 - j));
                stc<R>(dst + j, cscale(x, (R)k.cre));
            }
        }
    }

    // 1) kernel t_m at circular position p: m = min(p, L - p), and its DFT;
    // with one order for the whole batch the DFT is computed once (SPEC_WRITE)
    // and loaded by every signal (SPEC_READ), in natural order p = t + T e
    C<R> K[E];
    if constexpr (SREAD) {
        // the spectrum is read at the product below
    } else if (args.spec_mode == SPEC_READ) {
        const V *sp = reinterpret_cast<const V *>(args.spec);
#pragma unroll
        for (int e = 0; e < E; ++e)
            K[e] = ldc<R>(sp + t + T * e);
    } else {
        // m = p = t + T e for e < E/2, m = L - p = (N - t) - T (e - E/2) after
        // (the position p = N is never used by an output j < N)
        GaussSeq<R> lo(k.kmag, k.kph_hi, k.kph_lo, t, T), hi(k.kmag, k.kph_hi, k.kph_lo, N - t, -T);
#pragma unroll
        for (int e = 0; e < E; ++e)
            K[e] = e < E / 2 ? lo.next() : hi.next();
        fft_any<R, E, LFIX, DB>(K, lds, t, T, sc, lds1, &par);
        if (args.spec_mode == SPEC_WRITE) {
            // launched as one work-group; slot 0 holds the spectrum
            if (sl == 0) {
                V *sp = reinterpret_cast<V *>(args.spec);
#pragma unroll
                for (int e = 0; e < E; ++e)
                    stc<R>(sp + t + T * e, K[e]);
            }
            return;
        }
    }

    // 2) data e^{-P x_k^2} f_k (reversed for Hankel), zero-padded to L
    // (n_p = 2p - N + 1 = (2t - N + 1) + 2T e)
    C<R> v[E];
    {
        GaussSeq<R> dch(k.dmag, k.dph_hi, k.dph_lo, 2 * t - N + 1, 2 * T);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = t + T * e;
            C<R> x = {(R)0, (R)0};
            if (e < E / 2) { // p < N  <=>  e < E/2
                const C<R> w = dch.next();
                if (live && !k.special)
                    x = cmul(ldc<R>(src + (k.hankel ? N - 1 - p : p)), w);
            }
            v[e] = x;
        }
    }
    fft_any<R, E, LFIX, DB>(v, lds, t, T, sc, lds1, &par);

    // 3) inverse DFT of the product: conj(FFT(conj(V K)))
    if constexpr (SREAD) {
        const V *sp = reinterpret_cast<const V *>(args.spec);
#pragma unroll
        for (int e = 0; e < E; ++e)
            v[e] = cconj(cmul(v[e], ldc<R>(sp + t + T * e)));
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e)
            v[e] = cconj(cmul(v[e], K[e]));
    }
    fft_any<R, E, LFIX, DB>(v, lds, t, T, sc, lds1, &par);

    if (live && !k.special) {
        GaussSeq<R> och(k.omag, k.oph_hi, k.oph_lo, 2 * t - N + 1, 2 * T);
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int j = t + T * e;
            C<R> y = cconj(v[e]);
            y = cmul(y, och.next());
            y = cmul(y, C<R>{(R)k.cre, (R)k.cim});
            stc<R>(dst + j, y);
        }
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
template <typename R, int E, int NFIX, bool MF = false, int LB = max_block(sizeof(R) == 8, E), bool HX = false>
inline hipError_t launch_lct_t(const void *in, void *out, const LctArgs &a, int nblocks, int block, size_t lds,
                               hipStream_t s)
{
    auto kern = a.mode == MODE_FWD ? k_lct<R, E, NFIX, MODE_FWD, MF, LB, HX> : k_lct<R, E, NFIX, MODE_ADJ, MF, LB, HX>;
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(block), lds, s, (const typename Vec<R>::T *)in,
                       (typename Vec<R>::T *)out, a);
    return hipGetLastError();
}

// The forward transform storing only the window [a.win_off, a.win_off + a.win_n).
template <typename R, int E, int NFIX, int LB = max_block(sizeof(R) == 8, E)>
inline hipError_t launch_lct_window_t(const void *in, void *out, const LctArgs &a, int nblocks, int block, size_t lds,
                                      hipStream_t s)
{
    auto kern = k_lct<R, E, NFIX, MODE_FWD, false, LB, false, true>;
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(block), lds, s, (const typename Vec<R>::T *)in,
                       (typename Vec<R>::T *)out, a);
    return hipGetLastError();
}

template <typename R, int E, int NFIX = 0, int LB = max_block(sizeof(R) == 8, E)>
inline hipError_t launch_pgrad_t(const void *f, const void *g, double *grad4, const LctArgs &a, int nblocks,
                                 int block, size_t lds, hipStream_t s)
{
    auto kern = k_lct_pgrad<R, E, NFIX, LB>;
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(block), lds, s, (const typename Vec<R>::T *)f,
                       (const typename Vec<R>::T *)g, grad4, a);
    return hipGetLastError();
}

template <typename R, int E, int LFIX = 0, int LB = max_block(sizeof(R) == 8, E)>
inline hipError_t launch_frft_t(const void *in, void *out, const FrArgs &a, int nblocks, int block, size_t lds,
                                hipStream_t s)
{
    auto kern = k_frft<R, E, LFIX, LB>;
    if constexpr (LFIX > 0 && sizeof(R) == 8 && (E == 8 || E == 16)) {
        if (a.spec_mode == SPEC_READ)
            kern = k_frft<R, E, LFIX, LB, true>;
    }
    if constexpr (LFIX > 0 && sizeof(R) == 4) {
        if (a.spec_mode == SPEC_READ) {
            kern = k_frft<R, E, LFIX, LB, true>;
        } else if (LFIX == 8192 && a.S == 1) {
            // one work-group per CU by its registers: a second LDS buffer fits
            kern = k_frft<R, E, LFIX, LB, false, true>;
            lds *= 2;
        }
    }
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(block), lds, s, (const typename Vec<R>::T *)in,
                       (typename Vec<R>::T *)out, a);
    return hipGetLastError();
}


} // namespace lctk
