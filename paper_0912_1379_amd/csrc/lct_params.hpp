// lct_params.hpp - per-signal constants of the discrete LCT and of the
// same-grid fractional transform, derived from (a, b, c, d) or z in FP64
// (double-double where a phase coefficient multiplies n^2 up to 2^48).
// Shared by the host (plans) and the device (one matrix or order per signal).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace lctk {

// Error-free transformations: floating-point contraction is switched off in
// each of them, since fusing a product into a following sum would change the
// rounding these functions rely on.
struct DD {
    double hi, lo;
};

__host__ __device__ inline DD dd_two_prod(double a, double b)
{
#pragma clang fp contract(off)
    double p = a * b;
    return {p, fma(a, b, -p)};
}
__host__ __device__ inline DD dd_quick(double s, double e)
{
#pragma clang fp contract(off)
    double h = s + e;
    return {h, e - (h - s)};
}
__host__ __device__ inline DD dd_mul_d(DD x, double d)
{
#pragma clang fp contract(off)
    DD p = dd_two_prod(x.hi, d);
    return dd_quick(p.hi, fma(x.lo, d, p.lo));
}
__host__ __device__ inline DD dd_mul(DD x, DD y)
{
#pragma clang fp contract(off)
    DD p = dd_two_prod(x.hi, y.hi);
    return dd_quick(p.hi, p.lo + x.hi * y.lo + x.lo * y.hi);
}
__host__ __device__ inline DD dd_div_d(DD x, double d)
{
#pragma clang fp contract(off)
    double q1 = x.hi / d;
    DD r = dd_two_prod(q1, d);
    double rem = ((x.hi - r.hi) - r.lo) + x.lo;
    return dd_quick(q1, rem / d);
}

__host__ __device__ inline DD dd_two_sum(double a, double b)
{
#pragma clang fp contract(off)
    double s = a + b;
    double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ inline DD dd_add(DD x, DD y)
{
#pragma clang fp contract(off)
    DD s = dd_two_sum(x.hi, y.hi);
    return dd_quick(s.hi, s.lo + x.lo + y.lo);
}
__host__ __device__ inline DD dd_neg(DD x) { return {-x.hi, -x.lo}; }
__host__ __device__ inline DD dd_sub(DD x, DD y) { return dd_add(x, dd_neg(y)); }
__host__ __device__ inline DD dd_div(DD x, DD y)
{
#pragma clang fp contract(off)
    double q1 = x.hi / y.hi;
    DD r = dd_sub(x, dd_mul_d(y, q1));
    double q2 = r.hi / y.hi;
    return dd_quick(q1, q2);
}

// Complex double-double: the fractional and complex-matrix constants whose
// imaginary parts become phase coefficients per n^2 (up to 2^48 at the largest
// lengths) are formed in it, so that their rounding stays below the FP64
// transform's error.
struct CDD {
    DD re, im;
};
__host__ __device__ inline CDD cdd_mul(CDD a, CDD b)
{
    return {dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
}
__host__ __device__ inline CDD cdd_div(CDD a, CDD b)
{
    // a conj(b) / |b|^2, scaled by the larger part of b so that |b|^2 cannot overflow
    const double sc = fmax(fabs(b.re.hi), fabs(b.im.hi));
    const CDD bs{dd_div_d(b.re, sc), dd_div_d(b.im, sc)};
    const DD den = dd_add(dd_mul(bs.re, bs.re), dd_mul(bs.im, bs.im));
    const CDD num = cdd_mul(a, CDD{bs.re, dd_neg(bs.im)});
    return {dd_div_d(dd_div(num.re, den), sc), dd_div_d(dd_div(num.im, den), sc)};
}
__host__ __device__ inline CDD cdd_of(double re, double im) { return {DD{re, 0.0}, DD{im, 0.0}}; }

// pi and 1/(2 pi) as unevaluated double-double sums
constexpr double PI_HI = 3.141592653589793;
constexpr double PI_LO = 1.2246467991473532e-16;
constexpr double INV2PI_HI = 0.15915494309189535;
constexpr double INV2PI_LO = -9.839338337591243e-18;

// Per-signal constants of the LCT (Algorithm steps 1-2, b != 0), or of the
// b = 0 diagonal of §1.
//   pre:  turns per n_k^2 of the pre-chirp a x_k^2/(2b):   a pi / (32 b N)
//   post: turns per n_j^2 of the post-chirp d y_j^2/(2b):  b d / (2 pi N)
//   amp:  h (2 pi i b)^(-1/2) exp(-i pi (N-1)^2 / (2N))
// For b = 0: post holds c x_j^2/(2d) per n_j^2 (turns) and amp = sqrt(d).
// The amplitude is also kept in polar form (amp_mag, amp_turns) so that
// kernels can fold its phase into the post-chirp.
struct LctConst {
    double pre_hi, pre_lo;
    double post_hi, post_lo;
    double amp_re, amp_im;
    double amp_mag, amp_turns;
    int b0;
    int pad_;
};

__host__ __device__ inline LctConst lct_const(int64_t N, double a, double b, double c, double d)
{
    LctConst k{};
    if (b == 0.0) {
        // turns per n^2: c pi^2 n^2 / (8N) / (2d) / (2 pi) = c pi n^2 / (32 N d)
        DD t = dd_div_d(dd_div_d(dd_mul_d(DD{PI_HI, PI_LO}, c), d), 32.0 * (double)N);
        k.pre_hi = k.pre_lo = 0.0;
        k.post_hi = t.hi;
        k.post_lo = t.lo;
        if (d > 0) {
            k.amp_re = sqrt(d);
            k.amp_im = 0.0;
        } else {
            k.amp_re = 0.0;
            k.amp_im = sqrt(-d); // principal root of a negative number
        }
        k.amp_mag = sqrt(fabs(d));
        k.amp_turns = d > 0 ? 0.0 : 0.25;
        k.b0 = 1;
        return k;
    }
    // pre: a x^2/(2b) rad with x^2 = pi^2 n^2/(8N) -> a pi n^2 / (32 b N) turns
    DD pre = dd_div_d(dd_div_d(dd_mul_d(DD{PI_HI, PI_LO}, a), b), 32.0 * (double)N);
    // post: b d n^2 / N rad -> b d n^2 / (2 pi N) turns
    DD post = dd_div_d(dd_mul(dd_two_prod(b, d), DD{INV2PI_HI, INV2PI_LO}), (double)N);
    k.pre_hi = pre.hi;
    k.pre_lo = pre.lo;
    k.post_hi = post.hi;
    k.post_lo = post.lo;
    // h (2 pi i b)^(-1/2): principal root; 2 pi i b = 2 pi |b| e^{+-i pi/2}
    double h = PI_HI / sqrt(2.0 * (double)N);
    double mag = h / sqrt(2.0 * PI_HI * fabs(b));
    double ph = (b > 0) ? -0.125 : 0.125; // turns: e^{-+ i pi/4}
    // constant index phase -(N-1)^2/(4N) turns, reduced exactly
    int64_t m = (N - 1) * (N - 1) % (4 * N);
    ph -= (double)m / (4.0 * (double)N);
    ph -= rint(ph);
    k.amp_re = mag * cos(2.0 * PI_HI * ph);
    k.amp_im = mag * sin(2.0 * PI_HI * ph);
    k.amp_mag = mag;
    k.amp_turns = ph;
    k.b0 = 0;
    return k;
}

// Constants of the LCT that depend only on N, derived once on the host in
// extended precision so that a kernel holding one matrix per signal only
// needs a few FP64 operations per signal (lct_const_from):
//   pre:  pi / (32 N)   turns per n^2 and per unit of a/b
//   post: 1 / (2 pi N)  turns per n^2 and per unit of b d
//   hs:   h / sqrt(2 pi),  h = pi / sqrt(2N)
//   cpos/cneg: e^{-+i pi/4} e^{-i pi (N-1)^2/(2N)}, the phase of
//         h (2 pi i b)^(-1/2) e^{-i pi (N-1)^2/(2N)} for b > 0 / b < 0
struct NConst {
    double pre_hi, pre_lo;
    double post_hi, post_lo;
    double hs;
    double cpos_re, cpos_im;
    double cneg_re, cneg_im;
    double tpos, tneg; // the same two phases in turns
};

inline NConst n_const_host(int64_t N)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double n = (long double)N;
    NConst c{};
    long double pre = pi / (32.0L * n);
    long double post = 1.0L / (2.0L * pi * n);
    c.pre_hi = (double)pre;
    c.pre_lo = (double)(pre - (long double)c.pre_hi);
    c.post_hi = (double)post;
    c.post_lo = (double)(post - (long double)c.post_hi);
    c.hs = (double)((pi / sqrtl(2.0L * n)) / sqrtl(2.0L * pi));
    // constant index phase -(N-1)^2/(4N) turns, reduced exactly
    int64_t m = (N - 1) * (N - 1) % (4 * N);
    long double base = -(long double)m / (4.0L * n);
    long double tp = base - 0.125L, tn = base + 0.125L;
    c.cpos_re = (double)cosl(2.0L * pi * tp);
    c.cpos_im = (double)sinl(2.0L * pi * tp);
    c.cneg_re = (double)cosl(2.0L * pi * tn);
    c.cneg_im = (double)sinl(2.0L * pi * tn);
    c.tpos = (double)(tp - roundl(tp));
    c.tneg = (double)(tn - roundl(tn));
    return c;
}

// Per-signal LCT constants from the N-only constants: same values as
// lct_const, without transcendental functions.
__host__ __device__ inline LctConst lct_const_from(const NConst &nc, double a, double b, double c, double d)
{
    LctConst k{};
    const DD pre{nc.pre_hi, nc.pre_lo};
    if (b == 0.0) {
        // c x^2 / (2d) rad = c pi n^2 / (32 N d) turns
        DD t = dd_div_d(dd_mul_d(pre, c), d);
        k.post_hi = t.hi;
        k.post_lo = t.lo;
        k.amp_re = d > 0 ? sqrt(d) : 0.0;
        k.amp_im = d > 0 ? 0.0 : sqrt(-d);
        k.amp_mag = sqrt(fabs(d));
        k.amp_turns = d > 0 ? 0.0 : 0.25;
        k.b0 = 1;
        return k;
    }
    DD p = dd_div_d(dd_mul_d(pre, a), b);
    DD q = dd_mul_d(dd_mul_d(DD{nc.post_hi, nc.post_lo}, b), d);
    k.pre_hi = p.hi;
    k.pre_lo = p.lo;
    k.post_hi = q.hi;
    k.post_lo = q.lo;
    const double mag = nc.hs / sqrt(fabs(b));
    k.amp_re = mag * (b > 0 ? nc.cpos_re : nc.cneg_re);
    k.amp_im = mag * (b > 0 ? nc.cpos_im : nc.cneg_im);
    k.amp_mag = mag;
    k.amp_turns = b > 0 ? nc.tpos : nc.tneg;
    k.b0 = 0;
    return k;
}

// Validity of one signal's parameters (shared by the host checks and the
// device-side status check).
//   matrix (a, b, c, d): finite, and ad - bc = 1 (§1) within
//     |ad - bc - 1| <= 1e-10 max(1, |ad|, |bc|)  (this also excludes b = d = 0);
//   fractional order z: finite and |z| <= 1 + 1e-12 (eq. eqifft needs |z| <= 1;
//     the slack above 1 is projected onto the unit circle by fr_const).
__host__ __device__ inline bool lct_row_finite(double a, double b, double c, double d)
{
    return isfinite(a) && isfinite(b) && isfinite(c) && isfinite(d);
}
__host__ __device__ inline bool lct_row_unimodular(double a, double b, double c, double d)
{
    const double ad = a * d, bc = b * c;
    return fabs(ad - bc - 1.0) <= 1e-10 * fmax(1.0, fmax(fabs(ad), fabs(bc)));
}
__host__ __device__ inline bool frft_row_finite(double zr, double zi) { return isfinite(zr) && isfinite(zi); }
__host__ __device__ inline bool frft_row_in_disc(double zr, double zi) { return hypot(zr, zi) <= 1.0 + 1e-12; }

// Per-signal constants of the same-grid fractional transform (eq. fasy with
// y_j = x_j).  Writing the exponent as
//   -P (x_j^2 + x_k^2) - beta (x_j -+ x_k)^2
// with P = (1-z)/(2(1+z)), beta = z/(1-z^2) (Toeplitz, Re z >= 0) or
// P = (1+z)/(2(1-z)), beta = -z/(1-z^2) (Hankel, Re z < 0) makes Re P >= 0
// and Re beta >= 0, so every factor has modulus <= 1.
//   dmag/dph: log-modulus and turns of exp(-P x^2) per n^2 (x^2 = pi^2 n^2/(8N))
//   kmag/kph: log-modulus and turns of exp(-beta h^2 m^2) per m^2 (h^2 = pi^2/(2N))
//   cre/cim:  h sqrt(2/(1-z^2)) / L, L = 2N the convolution length
// special: 0 general, 1 for z = 1, 2 for z = -1 (continuum limits).
// Same-grid convolution form  out_j = C e^{o x_j^2} sum_k e^{kappa h^2 (j-k)^2} e^{d x_k^2} in'_k
// (in' = in, or in reversed for the Hankel form): log-modulus per n^2 and
// phase in turns per n^2 (double-double) of the input factor d and the output
// factor o (n = 2k - N + 1, x^2 = pi^2 n^2 / (8N)), and of the kernel per m^2;
// C includes the 1 / (2N) of the inverse DFT.  The fractional transform has
// o = d.
struct FrConst {
    double dmag, dph_hi, dph_lo;
    double kmag, kph_hi, kph_lo;
    double cre, cim;
    int hankel;
    int special;
    double omag, oph_hi, oph_lo;
};

__host__ __device__ inline void cdiv(double ar, double ai, double br, double bi, double &qr, double &qi)
{
    // Smith's algorithm
    if (fabs(br) >= fabs(bi)) {
        double r = bi / br, den = br + bi * r;
        qr = (ar + ai * r) / den;
        qi = (ai - ar * r) / den;
    } else {
        double r = br / bi, den = br * r + bi;
        qr = (ar * r + ai) / den;
        qi = (ai * r - ar) / den;
    }
}

__host__ __device__ inline void csqrt_principal(double re, double im, double &sr, double &si)
{
    double m = hypot(re, im);
    if (m == 0.0) {
        sr = si = 0.0;
        return;
    }
    if (re >= 0) {
        sr = sqrt(0.5 * (m + re));
        si = im / (2.0 * sr);
    } else {
        si = copysign(sqrt(0.5 * (m - re)), im);
        sr = im / (2.0 * si);
    }
}

// dd: P and beta in double-double (the host, and the FP64 kernels for
// per-signal orders); the FP32 kernels take them in double (their phase rates
// then carry a relative error of a few 1e-16, far below FP32 rounding, at a
// fraction of the cost: every thread forms its signal's constants).
__host__ __device__ inline FrConst fr_const(int64_t N, double zr, double zi, bool dd = true)
{
    FrConst k{};
    // orders accepted just outside the unit circle (|z| <= 1 + 1e-12) are
    // taken on it, where every factor still has modulus <= 1
    const double rz = hypot(zr, zi);
    if (rz > 1.0) {
        zr /= rz;
        zi /= rz;
    }
    if (zi == 0.0 && (zr == 1.0 || zr == -1.0)) {
        k.special = zr > 0 ? 1 : 2;
        k.cre = sqrt(2.0 * PI_HI);
        return k;
    }
    k.special = 0;
    k.hankel = zr < 0.0 ? 1 : 0;
    double s = k.hankel ? -1.0 : 1.0; // z -> s z maps the Hankel case onto the Toeplitz formulas
    double wr = s * zr, wi = s * zi;
    // P = (1 - w) / (2 (1 + w)), beta = w / (1 - w^2)  (w^2 = z^2); their
    // imaginary parts are phase rates per n^2 and m^2
    CDD P, B, om;
    if (dd) {
        P = cdd_div(CDD{dd_two_sum(1.0, -wr), DD{-wi, 0.0}}, CDD{dd_mul_d(dd_two_sum(1.0, wr), 2.0), DD{2.0 * wi, 0.0}});
        const CDD z2{dd_sub(dd_two_prod(zr, zr), dd_two_prod(zi, zi)), dd_mul_d(dd_two_prod(zr, zi), 2.0)};
        om = CDD{dd_sub(DD{1.0, 0.0}, z2.re), dd_neg(z2.im)};
        B = cdd_div(cdd_of(wr, wi), om);
    } else {
        double Pr, Pi, Br, Bi;
        cdiv(1.0 - wr, -wi, 2.0 * (1.0 + wr), 2.0 * wi, Pr, Pi);
        const double omr = 1.0 - (zr * zr - zi * zi), omi = -2.0 * zr * zi;
        cdiv(wr, wi, omr, omi, Br, Bi);
        P = cdd_of(Pr, Pi);
        B = cdd_of(Br, Bi);
        om = cdd_of(omr, omi);
    }
    const double n = (double)N;
    const DD pi{PI_HI, PI_LO};
    // exp(-P x^2), x^2 = pi^2 n^2 / (8N)
    k.dmag = -P.re.hi * PI_HI * PI_HI / (8.0 * n);
    DD dph = dd_div_d(dd_mul(pi, dd_neg(P.im)), 16.0 * n); // -Im P pi^2/(8N) / (2 pi)
    k.dph_hi = dph.hi;
    k.dph_lo = dph.lo;
    // exp(-beta h^2 m^2), h^2 = pi^2 / (2N)
    k.kmag = -B.re.hi * PI_HI * PI_HI / (2.0 * n);
    DD kph = dd_div_d(dd_mul(pi, dd_neg(B.im)), 4.0 * n); // -Im beta pi^2/(2N) / (2 pi)
    k.kph_hi = kph.hi;
    k.kph_lo = kph.lo;
    // h sqrt(2 / (1 - z^2)) / (2N)
    const double omr = om.re.hi + om.re.lo, omi = om.im.hi + om.im.lo;
    double qr, qi;
    cdiv(2.0, 0.0, omr, omi, qr, qi);
    double sr, si;
    csqrt_principal(qr, qi, sr, si);
    double h = PI_HI / sqrt(2.0 * n);
    k.cre = h * sr / (2.0 * n);
    k.cim = h * si / (2.0 * n);
    k.omag = k.dmag;
    k.oph_hi = k.dph_hi;
    k.oph_lo = k.dph_lo;
    return k;
}

} // namespace lctk
