// fft_core.hpp - device building blocks of the discrete LCT on gfx950:
// complex arithmetic, phase evaluation from turns reduced in FP64, small DFT
// butterflies, and a register-staged Stockham FFT held in LDS.
//
// The transform of the paper (Algorithm, eq. algfxft1) is a diagonal
// ("chirp-scaling") times a length-N DFT times a diagonal.  The DFT is
// computed here as a Stockham autosort FFT: each thread of a signal owns the E
// elements at positions t + T e (T = N / E threads per signal, e in [0, E)).
// Every stage reads exactly those positions, applies E / R radix-R butterflies
// in registers, and writes its outputs to the Stockham positions in LDS; the
// last stage's outputs land again on positions t + T e, so the first stage
// can read from HBM and the last stage can write to HBM directly, both
// coalesced across threads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lctk {

template <typename R> struct C {
    R x, y;
};

template <typename R> __device__ __forceinline__ C<R> cadd(C<R> a, C<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __device__ __forceinline__ C<R> csub(C<R> a, C<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __device__ __forceinline__ C<R> cmul(C<R> a, C<R> b)
{
    return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
template <typename R> __device__ __forceinline__ C<R> cconj(C<R> a) { return {a.x, -a.y}; }
template <typename R> __device__ __forceinline__ C<R> cscale(C<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by -i
template <typename R> __device__ __forceinline__ C<R> cmul_mi(C<R> a) { return {a.y, -a.x}; }
// multiply by +i
template <typename R> __device__ __forceinline__ C<R> cmul_pi(C<R> a) { return {-a.y, a.x}; }

// memory vector types: 8-byte complex64 / 16-byte complex128
template <typename R> struct Vec;
template <> struct Vec<float> { using T = float2; };
template <> struct Vec<double> { using T = double2; };

template <typename R> __device__ __forceinline__ C<R> ldc(const typename Vec<R>::T *p)
{
    typename Vec<R>::T v = *p;
    return {v.x, v.y};
}
template <typename R> __device__ __forceinline__ void stc(typename Vec<R>::T *p, C<R> a)
{
    typename Vec<R>::T v;
    v.x = a.x;
    v.y = a.y;
    *p = v;
}

// Buffer (descriptor-based) loads and stores: the base address and a byte
// limit live in scalar registers, the per-thread byte offset in a vector
// register and the per-element offset in a scalar register, so a strided
// sequence of accesses costs no vector address arithmetic.  Loads beyond the
// limit return zero and stores beyond it are dropped.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int BUF_DWORD3 = 0x00020000; // raw buffer, 32-bit data format (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, BUF_DWORD3);
}

template <typename R> struct Buf;
template <> struct Buf<float> {
    static __device__ __forceinline__ C<float> load(__amdgpu_buffer_rsrc_t r, int voff, int soff)
    {
        u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        return {__uint_as_float(v.x), __uint_as_float(v.y)};
    }
    static __device__ __forceinline__ void store(C<float> a, __amdgpu_buffer_rsrc_t r, int voff, int soff)
    {
        u32x2 v = {__float_as_uint(a.x), __float_as_uint(a.y)};
        __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
    }
};
template <> struct Buf<double> {
    static __device__ __forceinline__ C<double> load(__amdgpu_buffer_rsrc_t r, int voff, int soff)
    {
        u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        return {__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z)};
    }
    // The offset goes into the VGPR operand with a zero SGPR offset: with a
    // register soffset the compiler (ROCm 7.2) omits the wait state a
    // 128-bit store needs before its data VGPRs may be overwritten, and on
    // gfx950 the low dwords of some lanes were then stored from the next
    // value written to those registers.
    static __device__ __forceinline__ void store(C<double> a, __amdgpu_buffer_rsrc_t r, int voff, int soff)
    {
        unsigned long long x = (unsigned long long)__double_as_longlong(a.x);
        unsigned long long y = (unsigned long long)__double_as_longlong(a.y);
        u32x4 v = {(unsigned)x, (unsigned)(x >> 32), (unsigned)y, (unsigned)(y >> 32)};
        __builtin_amdgcn_raw_buffer_store_b128(v, r, voff + soff, 0, 0);
    }
};

// ---------------------------------------------------------------------------
// Phases.  A phase is carried in turns (1 turn = 2 pi rad), reduced to
// [-1/2, 1/2] in FP64, then evaluated as cos/sin(2 pi t) in the data precision.
// ---------------------------------------------------------------------------
// FP32: the hardware sine/cosine take their argument in turns; on |t| <= 1
// their error was measured at 1.3e-7 (max) / 4.9e-8 (rms) on gfx950, against
// 6.1e-8 / 2.1e-8 for the library's sincospif at about twenty times the cost.
__device__ __forceinline__ C<float> cis_turns(float t)
{
    return {__builtin_amdgcn_cosf(t), __builtin_amdgcn_sinf(t)};
}
__device__ __forceinline__ C<double> cis_turns(double t)
{
    double s, c;
    sincospi(2.0 * t, &s, &c);
    return {c, s};
}
template <typename R> __device__ __forceinline__ C<R> cis_turns_from(double t);
template <> __device__ __forceinline__ C<float> cis_turns_from<float>(double t) { return cis_turns((float)t); }
template <> __device__ __forceinline__ C<double> cis_turns_from<double>(double t) { return cis_turns(t); }

__device__ __forceinline__ double frac_turns(double t) { return t - rint(t); }

// Coefficient of a quadratic phase in turns, kept as an unevaluated sum
// hi + lo of two doubles (lo = 0 for the FP32 path, where one double suffices).
struct Quad {
    double hi, lo;
};

// frac(q * m2) for an exact integer m2 < 2^53 held in a double.
// Contraction must stay off here: fusing the product into the subtraction
// below would count its rounding error twice.
__device__ __forceinline__ double quad_turns(Quad q, double m2)
{
#pragma clang fp contract(off)
    double p = q.hi * m2;
    double e = fma(q.hi, m2, -p); // exact rounding error of the product
    double t = p - rint(p);
    return t + fma(q.lo, m2, e);
}

// Index phase of eq. (dislctn) with the integral's sign: (N-1) i / (2N) turns,
// reduced exactly: (N-1) i = N i - i and N i = N (i mod 2) (mod 2N).
__device__ __forceinline__ double index_turns(int i, int N, double inv2N)
{
    int r = (i & 1) ? (N - i) : (-i);
    return (double)r * inv2N;
}

// ---------------------------------------------------------------------------
// Small forward DFTs U_s = sum_r u_r exp(-2 pi i r s / R), in place.
// ---------------------------------------------------------------------------
template <typename R> struct K {
    static constexpr R SQH = (R)0.70710678118654752440084436210484904;  // sqrt(1/2)
    static constexpr R C8 = (R)0.92387953251128675612818318939678829;   // cos(pi/8)
    static constexpr R S8 = (R)0.38268343236508977172845998403039887;   // sin(pi/8)
    static constexpr R S3 = (R)0.86602540378443864676372317075293618;   // sin(pi/3)
    static constexpr R C5A = (R)0.30901699437494742410229341718281906;  // cos(2pi/5)
    static constexpr R C5B = (R)-0.80901699437494742410229341718281906; // cos(4pi/5)
    static constexpr R S5A = (R)0.95105651629515357211643933337938214;  // sin(2pi/5)
    static constexpr R S5B = (R)0.58778525229247312916870595463907277;  // sin(4pi/5)
};

template <typename R> __device__ __forceinline__ void dft2(C<R> &a, C<R> &b)
{
    C<R> t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <typename R> __device__ __forceinline__ void dft3(C<R> &a, C<R> &b, C<R> &c)
{
    C<R> s = cadd(b, c);
    C<R> d = csub(b, c);
    C<R> m = {a.x - (R)0.5 * s.x, a.y - (R)0.5 * s.y};
    C<R> r = cscale(cmul_mi(d), K<R>::S3); // -i sin(pi/3) (b - c)
    a = cadd(a, s);
    b = cadd(m, r);
    c = csub(m, r);
}

template <typename R> __device__ __forceinline__ void dft4(C<R> &a, C<R> &b, C<R> &c, C<R> &d)
{
    C<R> s0 = cadd(a, c), d0 = csub(a, c);
    C<R> s1 = cadd(b, d), d1 = cmul_mi(csub(b, d));
    a = cadd(s0, s1);
    c = csub(s0, s1);
    b = cadd(d0, d1);
    d = csub(d0, d1);
}

template <typename R> __device__ __forceinline__ void dft5(C<R> &u0, C<R> &u1, C<R> &u2, C<R> &u3, C<R> &u4)
{
    C<R> b1 = cadd(u1, u4), d1 = csub(u1, u4);
    C<R> b2 = cadd(u2, u3), d2 = csub(u2, u3);
    C<R> m1 = {u0.x + K<R>::C5A * b1.x + K<R>::C5B * b2.x, u0.y + K<R>::C5A * b1.y + K<R>::C5B * b2.y};
    C<R> m2 = {u0.x + K<R>::C5B * b1.x + K<R>::C5A * b2.x, u0.y + K<R>::C5B * b1.y + K<R>::C5A * b2.y};
    C<R> r1 = {K<R>::S5A * d1.x + K<R>::S5B * d2.x, K<R>::S5A * d1.y + K<R>::S5B * d2.y};
    C<R> r2 = {K<R>::S5B * d1.x - K<R>::S5A * d2.x, K<R>::S5B * d1.y - K<R>::S5A * d2.y};
    u0 = cadd(u0, cadd(b1, b2));
    C<R> i1 = cmul_mi(r1), i2 = cmul_mi(r2);
    u1 = cadd(m1, i1);
    u4 = csub(m1, i1);
    u2 = cadd(m2, i2);
    u3 = csub(m2, i2);
}

// radix 8 = 2 x 4
template <typename R> __device__ __forceinline__ void dft8(C<R> *u)
{
    dft4(u[0], u[2], u[4], u[6]);
    dft4(u[1], u[3], u[5], u[7]);
    // twiddles W8^p on the odd sub-transform
    u[3] = cmul(u[3], C<R>{K<R>::SQH, -K<R>::SQH});
    u[5] = cmul_mi(u[5]);
    u[7] = cmul(u[7], C<R>{-K<R>::SQH, -K<R>::SQH});
    C<R> o[8];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        C<R> e = u[2 * p], od = u[2 * p + 1];
        o[p] = cadd(e, od);
        o[p + 4] = csub(e, od);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s)
        u[s] = o[s];
}

// radix 16 = 4 x 4
template <typename R> __device__ __forceinline__ void dft16(C<R> *u)
{
#pragma unroll
    for (int q = 0; q < 4; ++q)
        dft4(u[q], u[q + 4], u[q + 8], u[q + 12]);
    // A_q[p] sits in u[q + 4p]; twiddle W16^(q p)
    const C<R> w1 = {K<R>::C8, -K<R>::S8}, w2 = {K<R>::SQH, -K<R>::SQH}, w3 = {K<R>::S8, -K<R>::C8};
    const C<R> w6 = {-K<R>::SQH, -K<R>::SQH}, w9 = {-K<R>::C8, K<R>::S8};
    u[1 + 4] = cmul(u[1 + 4], w1);
    u[1 + 8] = cmul(u[1 + 8], w2);
    u[1 + 12] = cmul(u[1 + 12], w3);
    u[2 + 4] = cmul(u[2 + 4], w2);
    u[2 + 8] = cmul_mi(u[2 + 8]);
    u[2 + 12] = cmul(u[2 + 12], w6);
    u[3 + 4] = cmul(u[3 + 4], w3);
    u[3 + 8] = cmul(u[3 + 8], w6);
    u[3 + 12] = cmul(u[3 + 12], w9);
    C<R> o[16];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        C<R> a = u[0 + 4 * p], b = u[1 + 4 * p], c = u[2 + 4 * p], d = u[3 + 4 * p];
        dft4(a, b, c, d);
        o[p] = a;
        o[p + 4] = b;
        o[p + 8] = c;
        o[p + 12] = d;
    }
#pragma unroll
    for (int s = 0; s < 16; ++s)
        u[s] = o[s];
}

template <int RAD, typename R> __device__ __forceinline__ void dft(C<R> *u)
{
    if constexpr (RAD == 2) {
        dft2(u[0], u[1]);
    } else if constexpr (RAD == 3) {
        dft3(u[0], u[1], u[2]);
    } else if constexpr (RAD == 4) {
        dft4(u[0], u[1], u[2], u[3]);
    } else if constexpr (RAD == 5) {
        dft5(u[0], u[1], u[2], u[3], u[4]);
    } else if constexpr (RAD == 8) {
        dft8(u);
    } else if constexpr (RAD == 16) {
        dft16(u);
    }
}

// Twiddles w^r = cis(r t0), r = 1..RAD-1.  FP32: the powers of two are
// evaluated directly (the hardware sine's error then enters each twiddle a
// few times at most instead of r times along a chain of products), the rest
// as one product of those.  FP64: w^1 from sincospi, the rest by products of
// depth <= 4 (sincospi in FP64 is accurate to an ulp, products add a few).
template <int RAD> __device__ __forceinline__ void twiddles(float t0, C<float> *w)
{
#pragma unroll
    for (int r = 1; r < RAD; r *= 2)
        w[r] = cis_turns((float)r * t0);
#pragma unroll
    for (int r = 3; r < RAD; ++r) {
        if ((r & (r - 1)) != 0) {
            const int hi = 1 << (31 - __builtin_clz(r));
            w[r] = cmul(w[hi], w[r - hi]);
        }
    }
}

template <int RAD> __device__ __forceinline__ void twiddles(double t0, C<double> *w);

// Twiddle powers w^r, r = 1..RAD-1, from w = w^1, with product depth <= 4.
template <int RAD, typename R> __device__ __forceinline__ void twiddle_powers(C<R> w1, C<R> *w)
{
    w[1] = w1;
    if constexpr (RAD > 2) w[2] = cmul(w1, w1);
    if constexpr (RAD > 3) w[3] = cmul(w[2], w1);
    if constexpr (RAD > 4) w[4] = cmul(w[2], w[2]);
    if constexpr (RAD > 5) {
#pragma unroll
        for (int r = 5; r < RAD && r < 8; ++r)
            w[r] = cmul(w[4], w[r - 4]);
    }
    if constexpr (RAD > 8) {
        w[8] = cmul(w[4], w[4]);
#pragma unroll
        for (int r = 9; r < RAD; ++r)
            w[r] = cmul(w[8], w[r - 8]);
    }
}

template <int RAD> __device__ __forceinline__ void twiddles(double t0, C<double> *w)
{
    twiddle_powers<RAD>(cis_turns(t0), w);
}

// Work-groups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remapping block i to logical index (i mod 8) * (n / 8) + i / 8 gives
// every XCD a contiguous range of logical tiles, so neighbouring tiles, which
// share cache lines, meet in one L2.  A bijection on the first 8 floor(n / 8)
// blocks, the identity on the rest.  Placement only: any mapping is correct.
__device__ __forceinline__ int xcd_remap(int i, int n)
{
    constexpr int X = 8;
    const int per = n / X;
    if (i >= per * X)
        return i;
    return (i % X) * per + i / X;
}

// a mod m for 0 <= a < 2^24 and m >= 1, with m the same in every lane (a stage
// stride, a transform length): a mask when m is a power of two; otherwise the
// quotient is estimated as trunc(a * rcp(m)) in FP32 and the remainder
// corrected exactly in integers.  The reciprocal (1 ulp) and the product (half
// an ulp) put the estimate within (a/m) 1.5 2^-23 < 1 of a/m for a < 2^24 and
// m >= 3, so one correction each way suffices; two are made below.  The
// generic 32-bit remainder is a sequence of about thirty instructions.
__device__ __forceinline__ int umod24(int a, int m)
{
    if ((m & (m - 1)) == 0)
        return a & (m - 1);
    const int q = (int)((float)a * __builtin_amdgcn_rcpf((float)m));
    int r = a - q * m;
    r += r < 0 ? m : 0;
    r += r < 0 ? m : 0;
    r -= r >= m ? m : 0;
    r -= r >= m ? m : 0;
    return r;
}

// LDS index with one pad element every 16 (breaks power-of-two bank strides).
__device__ __forceinline__ int lds_pad(int p) { return p + (p >> 4); }
__host__ __device__ constexpr int lds_elems(int N) { return N + (N >> 4) + 1; }

// a W16^k, W16 = e^{-2 pi i / 16}, for a compile-time k: the multiples of 4
// are free, the rest one product by a constant.
template <int k, typename R> __device__ __forceinline__ C<R> mul_w16(C<R> a)
{
    constexpr int m = k & 15;
    if constexpr (m >= 8) {
        const C<R> b = mul_w16<m - 8>(a);
        return C<R>{-b.x, -b.y};
    } else if constexpr (m >= 4) {
        return cmul_mi(mul_w16<m - 4>(a));
    } else if constexpr (m == 0) {
        return a;
    } else if constexpr (m == 1) {
        return cmul(a, C<R>{K<R>::C8, -K<R>::S8});
    } else if constexpr (m == 2) {
        return cmul(a, C<R>{K<R>::SQH, -K<R>::SQH});
    } else {
        return cmul(a, C<R>{K<R>::S8, -K<R>::C8});
    }
}

template <int E, int RAD, int I, int R0, typename R>
__device__ __forceinline__ void twiddles_shifted(const C<R> *w0, C<R> *w)
{
    if constexpr (R0 < RAD) {
        w[R0] = mul_w16<(I * R0 * (16 / E)) & 15>(w0[R0]);
        twiddles_shifted<E, RAD, I, R0 + 1>(w0, w);
    }
}

// Butterfly i's twiddles from butterfly 0's when T Q = Ns: positions b = t + T i
// do not wrap modulo Ns, so j_i = j_0 + T i and the base angle moves by
// -T i / (Ns RAD) = -i / E turns: w_i^r = w_0^r W_E^(i r).  E = 8 or 16.
template <int E, int RAD, int I, typename R> __device__ __forceinline__ void twiddles_next(const C<R> *w0, C<R> *w)
{
    twiddles_shifted<E, RAD, I, 1>(w0, w);
}

// One Stockham stage of radix RAD on the E register values of thread t.
// Input slot i + Q r (Q = E / RAD) holds position t + T (i + Q r); butterfly
// i has index b = t + T i and twiddle W_{Ns RAD}^{(b mod Ns) r}.  Outputs are
// left in place: slot i + Q s holds output s of butterfly i.
template <int E, int RAD, int I, typename R>
__device__ __forceinline__ void stage_compute_from(C<R> *v, int t, int T, int Ns, C<R> *w0)
{
    constexpr int Q = E / RAD;
    if constexpr (I < Q) {
        C<R> u[RAD];
#pragma unroll
        for (int r = 0; r < RAD; ++r)
            u[r] = v[I + Q * r];
        if (Ns > 1) {
            C<R> w[RAD];
            if constexpr (I > 0 && (E == 8 || E == 16)) {
                if (T * Q == Ns) {
                    twiddles_next<E, RAD, I>(w0, w);
                } else {
                    const int j = umod24(t + T * I, Ns);
                    twiddles<RAD>((R)(-j) * ((R)1 / (R)(Ns * RAD)), w);
                }
            } else {
                // base angle -j / (Ns RAD) turns (exact for power-of-two Ns RAD)
                const int j = umod24(t + T * I, Ns);
                twiddles<RAD>((R)(-j) * ((R)1 / (R)(Ns * RAD)), w);
                if constexpr (I == 0) {
#pragma unroll
                    for (int r = 1; r < RAD; ++r)
                        w0[r] = w[r];
                }
            }
#pragma unroll
            for (int r = 1; r < RAD; ++r)
                u[r] = cmul(u[r], w[r]);
        }
        dft<RAD>(u);
#pragma unroll
        for (int s = 0; s < RAD; ++s)
            v[I + Q * s] = u[s];
        stage_compute_from<E, RAD, I + 1>(v, t, T, Ns, w0);
    }
}

template <int E, int RAD, typename R>
__device__ __forceinline__ void stage_compute(C<R> *v, int t, int T, int Ns)
{
    C<R> w0[RAD];
    stage_compute_from<E, RAD, 0>(v, t, T, Ns, w0);
}

// What one LDS exchange moves: PART < 0 whole complex values (a C<R> array),
// PART = 0 / 1 only the real / imaginary parts (an R array, same indices).
template <int PART, typename R> struct LdsElem {
    using T = R;
};
template <typename R> struct LdsElem<-1, R> {
    using T = C<R>;
};
template <int PART, typename R> __device__ __forceinline__ typename LdsElem<PART, R>::T part_of(const C<R> &a)
{
    if constexpr (PART == 0)
        return a.x;
    else if constexpr (PART == 1)
        return a.y;
    else
        return a;
}
template <int PART, typename R> __device__ __forceinline__ void set_part(C<R> &a, const typename LdsElem<PART, R>::T &x)
{
    if constexpr (PART == 0)
        a.x = x;
    else if constexpr (PART == 1)
        a.y = x;
    else
        a = x;
}

// Writes the outputs of a stage to their Stockham positions in LDS.
// The padded index of p + s*d is lds_pad(p) + s*(d + d/16) when d is a
// multiple of 16, and lds_pad(p) + s*d when all of p + s*d stay inside one
// 16-element block; both keep one address per butterfly and constant offsets.
template <int E, int RAD, int PART = -1, typename R>
__device__ __forceinline__ void stage_write(typename LdsElem<PART, R>::T *lds, const C<R> *v, int t, int T, int Ns)
{
    constexpr int Q = E / RAD;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int b = t + T * i;
        int j = umod24(b, Ns);
        int base = (b - j) * RAD + j;
        auto *p = lds + lds_pad(base);
        if ((Ns & 15) == 0) {
            const int st = Ns + (Ns >> 4);
#pragma unroll
            for (int s = 0; s < RAD; ++s)
                p[s * st] = part_of<PART>(v[i + Q * s]);
        } else if ((base & 15) + (RAD - 1) * Ns < 16) {
#pragma unroll
            for (int s = 0; s < RAD; ++s)
                p[s * Ns] = part_of<PART>(v[i + Q * s]);
        } else {
#pragma unroll
            for (int s = 0; s < RAD; ++s)
                lds[lds_pad(base + s * Ns)] = part_of<PART>(v[i + Q * s]);
        }
    }
}

template <int E, int PART = -1, typename R>
__device__ __forceinline__ void stage_read(const typename LdsElem<PART, R>::T *lds, C<R> *v, int t, int T)
{
    if ((T & 15) == 0) {
        const auto *p = lds + lds_pad(t);
        const int st = T + (T >> 4);
#pragma unroll
        for (int e = 0; e < E; ++e)
            set_part<PART>(v[e], p[e * st]);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e)
            set_part<PART>(v[e], lds[lds_pad(t + T * e)]);
    }
}

template <int E, typename R>
__device__ __forceinline__ void run_stage(int rad, C<R> *v, int t, int T, int Ns)
{
    switch (rad) {
    case 16:
        if constexpr (E % 16 == 0) stage_compute<E, 16>(v, t, T, Ns);
        break;
    case 8:
        if constexpr (E % 8 == 0) stage_compute<E, 8>(v, t, T, Ns);
        break;
    case 5:
        if constexpr (E % 5 == 0) stage_compute<E, 5>(v, t, T, Ns);
        break;
    case 4:
        if constexpr (E % 4 == 0) stage_compute<E, 4>(v, t, T, Ns);
        break;
    case 3:
        if constexpr (E % 3 == 0) stage_compute<E, 3>(v, t, T, Ns);
        break;
    case 2:
        if constexpr (E % 2 == 0) stage_compute<E, 2>(v, t, T, Ns);
        break;
    default:
        break;
    }
}

template <int E, typename R>
__device__ __forceinline__ void run_write(int rad, C<R> *lds, const C<R> *v, int t, int T, int Ns)
{
    switch (rad) {
    case 16:
        if constexpr (E % 16 == 0) stage_write<E, 16>(lds, v, t, T, Ns);
        break;
    case 8:
        if constexpr (E % 8 == 0) stage_write<E, 8>(lds, v, t, T, Ns);
        break;
    case 5:
        if constexpr (E % 5 == 0) stage_write<E, 5>(lds, v, t, T, Ns);
        break;
    case 4:
        if constexpr (E % 4 == 0) stage_write<E, 4>(lds, v, t, T, Ns);
        break;
    case 3:
        if constexpr (E % 3 == 0) stage_write<E, 3>(lds, v, t, T, Ns);
        break;
    case 2:
        if constexpr (E % 2 == 0) stage_write<E, 2>(lds, v, t, T, Ns);
        break;
    default:
        break;
    }
}

// Radix schedule passed by value to kernels (stages in execution order).
// Kernels read it in place from their argument block (never copy it into a
// private array, which would live in scratch memory).
struct Sched {
    int nst;
    int rad[24];
};

// Radix of stage s of a compile-time schedule: greedy largest radix that
// divides both E and the remaining length.
__host__ __device__ constexpr int fixed_radix(int N, int E, int s)
{
    const int cand[6] = {16, 8, 5, 4, 3, 2};
    int rem = N;
    int r = 1;
    for (int k = 0; k <= s; ++k) {
        r = 1;
        for (int c = 0; c < 6; ++c) {
            if (E % cand[c] == 0 && rem % cand[c] == 0) {
                r = cand[c];
                break;
            }
        }
        rem /= r;
    }
    return r;
}
__host__ __device__ constexpr int fixed_nstages(int N, int E)
{
    int s = 0;
    while (s < 32 && fixed_radix(N, E, s) > 1)
        ++s;
    return s;
}

// True when a runtime schedule is the compile-time one of (N, E), so that a
// kernel instantiated for that length can run it.
__host__ __device__ inline bool is_fixed_sched(const Sched &sc, int N, int E)
{
    if (sc.nst != fixed_nstages(N, E))
        return false;
    for (int s = 0; s < sc.nst; ++s)
        if (sc.rad[s] != fixed_radix(N, E, s))
            return false;
    return true;
}

// In-LDS forward FFT of the register values v (positions t + T e), in place.
// All threads of the work-group must call it (it contains barriers).  On
// return v[e] holds output position t + T e.  The LDS buffer is free again
// after the first barrier of the next call.
// Compile-time schedule version: every stage's radix and stride are constants.
template <int E, int N, int S, int NS, typename R>
__device__ __forceinline__ void fft_lds_fixed_from(C<R> *v, C<R> *lds, int t)
{
    constexpr int NST = fixed_nstages(N, E);
    if constexpr (S < NST) {
        constexpr int RAD = fixed_radix(N, E, S);
        constexpr int T = N / E;
        stage_compute<E, RAD>(v, t, T, NS);
        if constexpr (S + 1 < NST) {
            __syncthreads();
            stage_write<E, RAD>(lds, v, t, T, NS);
            __syncthreads();
            stage_read<E>(lds, v, t, T);
        }
        fft_lds_fixed_from<E, N, S + 1, NS * RAD>(v, lds, t);
    }
}
template <int E, int N, typename R>
__device__ __forceinline__ void fft_lds_fixed(C<R> *v, C<R> *lds, int t)
{
    fft_lds_fixed_from<E, N, 0, 1>(v, lds, t);
}

// Same transform with the exchanges alternating between two LDS buffers.
// Exchange k writes buffer k mod 2, waits at one barrier and reads it back:
// the buffer it overwrites was last read in exchange k - 2, and every thread
// finished that read before writing exchange k - 1, i.e. before the barrier
// of exchange k - 1 that this thread has passed.  One barrier per stage
// instead of two.  `par` carries the alternation across calls (start it at 0
// and pass the same variable to every FFT of the kernel).
template <int E, int N, int S, int NS, typename R>
__device__ __forceinline__ void fft_lds_fixed2_from(C<R> *v, C<R> *lds0, C<R> *lds1, int t, int &par)
{
    constexpr int NST = fixed_nstages(N, E);
    if constexpr (S < NST) {
        constexpr int RAD = fixed_radix(N, E, S);
        constexpr int T = N / E;
        stage_compute<E, RAD>(v, t, T, NS);
        if constexpr (S + 1 < NST) {
            C<R> *buf = par ? lds1 : lds0;
            par ^= 1;
            stage_write<E, RAD>(buf, v, t, T, NS);
            __syncthreads();
            stage_read<E>(buf, v, t, T);
        }
        fft_lds_fixed2_from<E, N, S + 1, NS * RAD>(v, lds0, lds1, t, par);
    }
}
template <int E, int N, typename R>
__device__ __forceinline__ void fft_lds_fixed2(C<R> *v, C<R> *lds0, C<R> *lds1, int t, int &par)
{
    fft_lds_fixed2_from<E, N, 0, 1>(v, lds0, lds1, t, par);
}

// Same transform with each exchange made in two halves, the real parts and
// then the imaginary parts, through a buffer of lds_elems(N) R (half the LDS
// of the whole-value exchange, for two more barriers per stage).
template <int E, int N, int S, int NS, typename R>
__device__ __forceinline__ void fft_lds_fixed_half_from(C<R> *v, R *lds, int t)
{
    constexpr int NST = fixed_nstages(N, E);
    if constexpr (S < NST) {
        constexpr int RAD = fixed_radix(N, E, S);
        constexpr int T = N / E;
        stage_compute<E, RAD>(v, t, T, NS);
        if constexpr (S + 1 < NST) {
            // reading the real parts leaves the imaginary parts of the stage's
            // outputs in place for the second half
            __syncthreads();
            stage_write<E, RAD, 0>(lds, v, t, T, NS);
            __syncthreads();
            stage_read<E, 0>(lds, v, t, T);
            __syncthreads();
            stage_write<E, RAD, 1>(lds, v, t, T, NS);
            __syncthreads();
            stage_read<E, 1>(lds, v, t, T);
        }
        fft_lds_fixed_half_from<E, N, S + 1, NS * RAD>(v, lds, t);
    }
}
template <int E, int N, typename R>
__device__ __forceinline__ void fft_lds_fixed_half(C<R> *v, R *lds, int t)
{
    fft_lds_fixed_half_from<E, N, 0, 1>(v, lds, t);
}

template <int E, typename R>
__device__ __forceinline__ void fft_lds(C<R> *v, C<R> *lds, int t, int T, const Sched &sc)
{
    int Ns = 1;
    for (int s = 0; s < sc.nst; ++s) {
        const int rad = sc.rad[s];
        run_stage<E>(rad, v, t, T, Ns);
        if (s + 1 < sc.nst) {
            __syncthreads(); // previous readers of lds are done
            run_write<E>(rad, lds, v, t, T, Ns);
            __syncthreads();
            stage_read<E>(lds, v, t, T);
        }
        Ns *= rad;
    }
}

} // namespace lctk
