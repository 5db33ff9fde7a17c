// lct_api.hip - host side of the C ABI declared in include/lct.h: argument
// validation, plan constants, size/tiling selection and kernel dispatch.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include <complex>
#include <mutex>
#include <new>

#include "../../include/lct.h"
#include "plan.hpp"

using namespace lctk;

struct lct_plan_s {
    int64_t N;
    int prec;
    double a, b, c, d;
    double s; // input grid scale: samples on s x_k
    LctConst k;
};

namespace {

int fs_run(int64_t N, bool fp64, bool mf, const double *M4, const LctConst *k, int mode, const void *in, void *out,
           int64_t batch, hipStream_t s)
{
    if (in == out)
        return LCT_ERR_ARG; // pass 1 reads columns of `in` while writing rows of `out`
    const FsTiling f = mf ? mfma_fs(N) : select_fs(LCT_TUNE_LCT, N, N, fp64);
    if (!f.ok)
        return LCT_ERR_UNSUPPORTED;
    return fs_launch(f, N, fp64, M4, k, mode, in, out, batch, s);
}

int check_ptr(const void *p, bool fp64)
{
    if (p == nullptr)
        return LCT_ERR_ARG;
    if (((uintptr_t)p) % (fp64 ? 16 : 8) != 0)
        return LCT_ERR_ARG;
    return LCT_OK;
}

int validate_M(double a, double b, double c, double d)
{
    if (!lct_row_finite(a, b, c, d))
        return LCT_ERR_ARG;
    if (!lct_row_unimodular(a, b, c, d))
        return LCT_ERR_NOT_UNIMODULAR;
    return LCT_OK;
}

int validate_z(double z_re, double z_im)
{
    if (!frft_row_finite(z_re, z_im))
        return LCT_ERR_ARG;
    if (!frft_row_in_disc(z_re, z_im))
        return LCT_ERR_DOMAIN;
    return LCT_OK;
}

// Constants of the transform of samples taken on the input grid xi_k = s x_k
// (s > 0), outputs at y_j = 4 b x_j / (pi s) for b != 0 and xi_j / d for b = 0.
// The Riemann sum of the integral of §1 on that grid keeps the cross phase
// xi_k y_j / b = pi n_j n_k / (2N) (still a DFT) and changes
//   pre  a xi_k^2 / (2b) = a s^2 pi^2 n_k^2 / (16 b N) rad
//   post d y_j^2 / (2b)  = b d n_j^2 / (N s^2) rad
//   amplitude            s h (2 pi i b)^(-1/2)  (the quadrature weight is s h)
// and for b = 0 the chirp c xi_j^2 / (2d) = c s^2 pi^2 n_j^2 / (16 N d) rad with
// the amplitude sqrt(d) unchanged.  Coefficients in double-double as in
// lct_const, so s costs no precision; s == 1 is lct_const itself.
LctConst lct_const_scaled(int64_t N, double a, double b, double c, double d, double s)
{
    LctConst k = lct_const(N, a, b, c, d);
    if (s == 1.0)
        return k;
    const DD pi{PI_HI, PI_LO};
    if (b == 0.0) {
        const DD t = dd_div_d(dd_div_d(dd_mul_d(dd_mul_d(dd_mul_d(pi, c), s), s), d), 32.0 * (double)N);
        k.post_hi = t.hi;
        k.post_lo = t.lo;
        return k;
    }
    const DD pre = dd_div_d(dd_div_d(dd_mul_d(dd_mul_d(dd_mul_d(pi, a), s), s), b), 32.0 * (double)N);
    const DD post =
        dd_div_d(dd_div_d(dd_div_d(dd_mul(dd_two_prod(b, d), DD{INV2PI_HI, INV2PI_LO}), (double)N), s), s);
    k.pre_hi = pre.hi;
    k.pre_lo = pre.lo;
    k.post_hi = post.hi;
    k.post_lo = post.lo;
    k.amp_re *= s;
    k.amp_im *= s;
    k.amp_mag *= s;
    return k;
}

bool lct_const_finite(const LctConst &k)
{
    return isfinite(k.pre_hi) && isfinite(k.pre_lo) && isfinite(k.post_hi) && isfinite(k.post_lo) &&
           isfinite(k.amp_mag) && k.amp_mag > 0.0;
}

int lct_run(int64_t N, bool fp64, bool mf, const double *M4, const LctConst *k, int mode, const void *in, void *out,
            int64_t batch, hipStream_t s)
{
    if (batch < 0)
        return LCT_ERR_ARG;
    if (!smooth235(N))
        return LCT_ERR_UNSUPPORTED_N;
    if (batch == 0)
        return LCT_OK;
    int rc;
    if ((rc = check_ptr(in, fp64)) || (rc = check_ptr(out, fp64)))
        return rc;
    if (N > single_pass_limit(fp64))
        return fs_run(N, fp64, mf, M4, k, mode, in, out, batch, s);
    const Tiling tl = mf ? mfma_tiling(N) : select_tiling(LCT_TUNE_LCT, N, N, fp64, 0);
    if (!tl.ok)
        return LCT_ERR_UNSUPPORTED;
    return lct_launch(tl, N, fp64, M4, k, mode, in, out, batch, s);
}

// Single pass: room for the kernel spectrum of a shared order (2N complex
// values; optional, used by frft_exec_ws).  Two passes: data and kernel
// regions of 2N complex values per signal (required).
size_t frft_ws_bytes(int64_t N, bool fp64, int64_t batch)
{
    if (2 * N <= single_pass_limit(fp64))
        return (size_t)(2 * N) * (fp64 ? 16 : 8);
    return (size_t)batch * 2 * (size_t)(2 * N) * (fp64 ? 16 : 8);
}

// Constants of the same-grid LCT of a complex matrix (a, b, d; b != 0): the
// Riemann sum of the integral of §1 with y_j = x_j,
//   G_j = h (2 pi i b)^(-1/2) sum_k exp(w [a x_k^2 - 2 x_k x_j + d x_j^2]) f_k,  w = i / (2b),
// split exactly with -2 x_k x_j = (x_j - x_k)^2 - x_j^2 - x_k^2 (Toeplitz:
// input factor w (a - 1), kernel w, output factor w (d - 1)) or
// -2 x_k x_j = -(x_j + x_k)^2 + x_j^2 + x_k^2 (Hankel, the input reversed so
// that x_j + x_k = x_j - x_k': input factor w (a + 1), kernel -w, output
// factor w (d + 1)).  The form whose three factors all have non-positive
// real parts (every factor of modulus <= 1) is taken, Toeplitz first;
// neither gives LCT_ERR_DOMAIN.
int same_grid_const(int64_t N, double ar, double ai, double br, double bi, double dr, double di, FrConst *k)
{
    // w = i / (2b) and the factors in double-double: their imaginary parts
    // become phase rates per n^2
    const CDD w = cdd_div(cdd_of(0.0, 1.0), cdd_of(2.0 * br, 2.0 * bi));
    auto mulw = [&](double xr, double sgn, double xi) { return cdd_mul(w, CDD{dd_two_sum(xr, sgn), DD{xi, 0.0}}); };
    auto bounded = [](const CDD &x) { return x.re.hi <= 1e-12 * fmax(1.0, fabs(x.im.hi)); };
    const CDD ti = mulw(ar, -1.0, ai), to = mulw(dr, -1.0, di);
    const CDD hi = mulw(ar, 1.0, ai), ho = mulw(dr, 1.0, di);
    const CDD wn{dd_neg(w.re), dd_neg(w.im)};
    const bool toep = bounded(ti) && bounded(w) && bounded(to);
    const bool hank = bounded(hi) && bounded(wn) && bounded(ho);
    if (!toep && !hank)
        return LCT_ERR_DOMAIN;
    *k = FrConst{};
    k->special = 0;
    k->hankel = toep ? 0 : 1;
    const CDD in = toep ? ti : hi, ou = toep ? to : ho, kk = toep ? w : wn;
    const double n = (double)N;
    const DD pi{PI_HI, PI_LO};
    // x^2 = pi^2 n^2 / (8N): log-modulus Re(.) pi^2 / (8N), turns Im(.) pi / (16N) per n^2
    k->dmag = in.re.hi * PI_HI * PI_HI / (8.0 * n);
    DD t = dd_div_d(dd_mul(pi, in.im), 16.0 * n);
    k->dph_hi = t.hi;
    k->dph_lo = t.lo;
    k->omag = ou.re.hi * PI_HI * PI_HI / (8.0 * n);
    t = dd_div_d(dd_mul(pi, ou.im), 16.0 * n);
    k->oph_hi = t.hi;
    k->oph_lo = t.lo;
    // h^2 m^2 = pi^2 m^2 / (2N): log-modulus Re pi^2 / (2N), turns Im pi / (4N) per m^2
    k->kmag = kk.re.hi * PI_HI * PI_HI / (2.0 * n);
    t = dd_div_d(dd_mul(pi, kk.im), 4.0 * n);
    k->kph_hi = t.hi;
    k->kph_lo = t.lo;
    // h (2 pi i b)^(-1/2) / (2N), principal root; 2 pi i b = -2 pi b_im + i 2 pi b_re
    double sr, si;
    csqrt_principal(-2.0 * PI_HI * bi, 2.0 * PI_HI * br, sr, si);
    double qr, qi;
    cdiv(1.0, 0.0, sr, si, qr, qi);
    const double h = PI_HI / sqrt(2.0 * n);
    k->cre = h * qr / (2.0 * n);
    k->cim = h * qi / (2.0 * n);
    return LCT_OK;
}

// Constants of the complex-matrix LCT at the complex nodes y_j = 4 b x_j / pi
// (cx_impl.hpp).  With x^2 = pi^2 n^2 / (8N):
//   pre  exp(i a x^2/(2b)):  log-modulus -Im(a/b) pi^2 / (16N), turns Re(a/b) pi / (32N) per n^2
//   post exp(i d y^2/(2b)) = exp(i b d n^2 / N):  log-modulus -Im(bd) / N, turns Re(bd) / (2 pi N)
//   amp  h (2 pi i b)^(-1/2) e^{-i pi (N-1)^2 / (2N)}  (principal root)
// a/b and bd in double-double (their parts multiply n^2).  Both diagonals
// must have modulus <= 1: Im(a/b) >= 0 and Im(bd) >= 0 (relative slack
// 1e-12), else LCT_ERR_DOMAIN.
int cx_const(int64_t N, double ar, double ai, double br, double bi, double dr, double di, CxConst *k)
{
    const CDD A = cdd_of(ar, ai), B = cdd_of(br, bi), D = cdd_of(dr, di);
    const CDD ab = cdd_div(A, B), bd = cdd_mul(B, D);
    if (ab.im.hi < -1e-12 * fmax(1.0, fabs(ab.re.hi)) || bd.im.hi < -1e-12 * fmax(1.0, fabs(bd.re.hi)))
        return LCT_ERR_DOMAIN;
    const double n = (double)N;
    *k = CxConst{};
    k->pre_mag = -fmax(ab.im.hi, 0.0) * PI_HI * PI_HI / (16.0 * n);
    DD t = dd_div_d(dd_mul(DD{PI_HI, PI_LO}, ab.re), 32.0 * n);
    k->pre_hi = t.hi;
    k->pre_lo = t.lo;
    k->post_mag = -fmax(bd.im.hi, 0.0) / n;
    t = dd_div_d(dd_mul(bd.re, DD{INV2PI_HI, INV2PI_LO}), n);
    k->post_hi = t.hi;
    k->post_lo = t.lo;
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double h = pi / sqrtl(2.0L * (long double)N);
    using cld = std::complex<long double>;
    const cld root = std::sqrt(cld(0.0L, 2.0L * pi) * cld((long double)br, (long double)bi)); // principal
    const int64_t m = (N - 1) * (N - 1) % (4 * N);
    const cld amp = h / root * std::exp(cld(0.0L, -pi * (long double)m / (2.0L * (long double)N)));
    k->amp_re = (double)amp.real();
    k->amp_im = (double)amp.imag();
    if (!isfinite(k->pre_mag) || !isfinite(k->pre_hi) || !isfinite(k->post_mag) || !isfinite(k->post_hi) ||
        !isfinite(k->amp_re) || !isfinite(k->amp_im))
        return LCT_ERR_ARG;
    return LCT_OK;
}

int frft_run(int64_t N, bool fp64, const double *Z2, const FrConst *k, const void *in, void *out, int64_t batch,
             void *ws, size_t ws_bytes, hipStream_t s)
{
    if (batch < 0)
        return LCT_ERR_ARG;
    if (!smooth235(N))
        return LCT_ERR_UNSUPPORTED_N;
    if (batch == 0)
        return LCT_OK;
    int rc;
    if ((rc = check_ptr(in, fp64)) || (rc = check_ptr(out, fp64)))
        return rc;
    if (in == out)
        return LCT_ERR_ARG; // the Hankel form reads the input reversed
    if (2 * N > single_pass_limit(fp64)) {
        const size_t need = frft_ws_bytes(N, fp64, batch);
        if (ws == nullptr || ws_bytes < need || ((uintptr_t)ws) % 16)
            return LCT_ERR_WORKSPACE;
        const FsTiling f = select_fs(LCT_TUNE_FRFT, N, 2 * N, fp64);
        if (!f.ok)
            return LCT_ERR_UNSUPPORTED;
        return frft_large_launch(f, N, fp64, Z2, k, in, out, batch, ws, s);
    }
    const Tiling tl = select_tiling(LCT_TUNE_FRFT, N, 2 * N, fp64, 0);
    if (!tl.ok)
        return LCT_ERR_UNSUPPORTED;
    // one order for the whole batch and room for its spectrum: transform the
    // kernel once instead of once per signal
    void *spec = nullptr;
    if (Z2 == nullptr && ws != nullptr && ws_bytes >= frft_ws_bytes(N, fp64, batch) && ((uintptr_t)ws) % 16 == 0)
        spec = ws;
    return frft_sp_launch(tl, N, fp64, Z2, k, in, out, batch, s, spec);
}

} // namespace

namespace lctk {

int hip_status(hipError_t e) { return e == hipSuccess ? LCT_OK : LCT_ERR_HIP; }

int lct_launch(const Tiling &tl, int64_t N, bool fp64, const double *M4, const LctConst *k, int mode, const void *in,
               void *out, int64_t batch, hipStream_t s)
{
    LctArgs a{};
    a.N = (int)N;
    a.T = tl.T;
    a.S = tl.S;
    a.mode = mode;
    a.batch = batch;
    a.M4 = M4;
    if (k)
        a.k = *k;
    a.nc = n_const_host(N);
    a.sc = tl.sc;
    const int64_t nb = (batch + tl.S - 1) / tl.S;
    if (nb > INT32_MAX)
        return LCT_ERR_ARG;
    if (tl.mf)
        return hip_status(launch_lct_mf(in, out, a, (int)nb, tl.block, tl.lds, s));
    return hip_status(launch_lct(fp64, tl.E, in, out, a, (int)nb, tl.block, tl.lds, s));
}

// Single-pass forward transform of length N storing only the outputs
// [off, off + n) of each signal, n per signal at out; LCT_ERR_UNSUPPORTED
// where the geometry has no windowed instantiation (the caller then
// transforms in full and copies the window).
int lct_launch_window(int64_t N, bool fp64, const LctConst *k, const void *in, void *out, int64_t batch, int off,
                      int n, hipStream_t s)
{
    const Tiling tl = select_tiling(LCT_TUNE_LCT, N, N, fp64, 0);
    if (!tl.ok || tl.mf || tl.S != 1)
        return LCT_ERR_UNSUPPORTED;
    LctArgs a{};
    a.N = (int)N;
    a.T = tl.T;
    a.S = tl.S;
    a.mode = 0;
    a.batch = batch;
    a.k = *k;
    a.nc = n_const_host(N);
    a.sc = tl.sc;
    a.win_off = off;
    a.win_n = n;
    if (batch > INT32_MAX)
        return LCT_ERR_ARG;
    const hipError_t e = launch_lct_window(fp64, tl.E, in, out, a, (int)batch, tl.block, tl.lds, s);
    return e == hipErrorNotSupported ? LCT_ERR_UNSUPPORTED : hip_status(e);
}

int fs_launch(const FsTiling &f, int64_t N, bool fp64, const double *M4, const LctConst *k, int mode, const void *in,
              void *out, int64_t batch, hipStream_t s)
{
    FsArgs a{};
    a.N = (int)N;
    a.N1 = f.N1;
    a.N2 = f.N2;
    a.C = f.C;
    a.RR = f.RR;
    a.T1 = f.T1;
    a.T2 = f.T2;
    a.mode = mode;
    a.batch = batch;
    a.M4 = M4;
    if (k)
        a.k = *k;
    a.nc = n_const_host(N);
    a.sc1 = f.sc1;
    a.sc2 = f.sc2;
    const int64_t nb1 = batch * (f.N2 / f.C), nb2 = batch * (f.N1 / f.RR);
    if (nb1 > INT32_MAX || nb2 > INT32_MAX)
        return LCT_ERR_ARG;
    hipError_t e = f.mf1 ? launch_fs1_mf(in, out, a, (int)nb1, f.bs1, f.lds1, s)
                         : launch_fs1(fp64, f.E1, in, out, a, (int)nb1, f.bs1, f.lds1, s);
    if (e != hipSuccess)
        return LCT_ERR_HIP;
    return hip_status(f.mf2 ? launch_fs2_mf(out, a, (int)nb2, f.bs2, f.lds2, s)
                            : launch_fs2(fp64, f.E2, out, a, (int)nb2, f.bs2, f.lds2, s));
}

int frft_sp_launch(const Tiling &tl, int64_t N, bool fp64, const double *Z2, const FrConst *k, const void *in,
                   void *out, int64_t batch, hipStream_t s, void *spec)
{
    FrArgs a{};
    a.N = (int)N;
    a.T = tl.T;
    a.S = tl.S;
    a.batch = batch;
    a.Z2 = Z2;
    if (k)
        a.k = *k;
    a.sc = tl.sc;
    const int64_t nb = (batch + tl.S - 1) / tl.S;
    if (nb > INT32_MAX)
        return LCT_ERR_ARG;
    if (spec != nullptr && Z2 == nullptr && k != nullptr && !k->special) {
        // the kernel's spectrum once: one work-group, one slot
        FrArgs w = a;
        w.S = 1;
        w.batch = 1;
        w.spec_mode = SPEC_WRITE;
        w.spec = spec;
        const size_t lds1 = (size_t)lds_elems((int)(2 * N)) * (fp64 ? 16 : 8);
        hipError_t e = launch_frft(fp64, tl.E, in, out, w, 1, tl.T, lds1, s);
        if (e != hipSuccess)
            return LCT_ERR_HIP;
        a.spec_mode = SPEC_READ;
        a.spec = spec;
    }
    return hip_status(launch_frft(fp64, tl.E, in, out, a, (int)nb, tl.block, tl.lds, s));
}

int frft_large_launch(const FsTiling &f, int64_t N, bool fp64, const double *Z2, const FrConst *k, const void *in,
                      void *out, int64_t batch, void *ws, hipStream_t s)
{
    FrLArgs a{};
    a.N = (int)N;
    a.L = (int)(2 * N);
    a.L1 = f.N1;
    a.L2 = f.N2;
    a.C = f.C;
    a.RR = f.RR;
    a.T1 = f.T1;
    a.T2 = f.T2;
    a.batch = batch;
    a.Z2 = Z2;
    if (k)
        a.k = *k;
    a.sc1 = f.sc1;
    a.sc2 = f.sc2;
    const int64_t nb1 = batch * (f.N2 / f.C), nb2 = batch * (f.N1 / f.RR);
    if (2 * nb1 > INT32_MAX || nb2 > INT32_MAX || batch > INT32_MAX)
        return LCT_ERR_ARG;
    // one order for the batch: the kernel sequence is transformed once (its
    // column pass for slot 0 only, then its row pass in place there)
    const bool shared = Z2 == nullptr && k != nullptr && !k->special;
    const int64_t nk1 = shared ? f.N2 / f.C : nb1;
    hipError_t e;
    if ((e = launch_frl1(fp64, f.E1, in, ws, a, (int)(nb1 + nk1), f.bs1, f.lds1, s)) != hipSuccess)
        return LCT_ERR_HIP;
    if (shared) {
        FrLArgs w = a;
        w.spec_mode = SPEC_WRITE;
        if ((e = launch_frl2(fp64, f.E2, ws, w, f.N1 / f.RR, f.bs2, f.lds2, s)) != hipSuccess)
            return LCT_ERR_HIP;
        a.spec_mode = SPEC_READ;
    }
    if ((e = launch_frl2(fp64, f.E2, ws, a, (int)nb2, f.bs2, f.lds2, s)) != hipSuccess ||
        (e = launch_frl3(fp64, f.E1, ws, out, a, (int)nb1, f.bs1, f.lds1, s)) != hipSuccess)
        return LCT_ERR_HIP;
    if (Z2 != nullptr || (k && k->special))
        return hip_status(launch_fr_special(fp64, in, out, a, s));
    return LCT_OK;
}

} // namespace lctk

namespace {

// Workspace of frft_exec_noalloc: one array per device, held until the process
// ends.  In host code `scratch` only names the symbol; its device address comes
// from hipGetSymbolAddress, once per device with that device current.
__device__ __align__(256) unsigned char scratch[LCT_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 256;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES];

int scratch_of_current_device(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return LCT_ERR_HIP;
    if (dev < 0 || dev >= MAX_DEVICES)
        return LCT_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> g(scratch_mu);
    if (scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return LCT_ERR_HIP;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return LCT_OK;
}

} // namespace

extern "C" {

int64_t lct_max_single_pass(lct_precision prec) { return single_pass_limit(prec == LCT_FP64); }

int lct_plan_create_ex(lct_plan *out, int64_t N, double a, double b, double c, double d, lct_precision prec)
{
    if (out == nullptr)
        return LCT_ERR_ARG;
    *out = nullptr;
    if (prec != LCT_FP32 && prec != LCT_FP64 && prec != LCT_FP32_SPLITBF16)
        return LCT_ERR_ARG;
    if (!smooth235(N))
        return LCT_ERR_UNSUPPORTED_N;
    int rc = validate_M(a, b, c, d);
    if (rc)
        return rc;
    if (b == 0.0 && d == 0.0)
        return LCT_ERR_NOT_UNIMODULAR;
    lct_plan p = new (std::nothrow) lct_plan_s;
    if (!p)
        return LCT_ERR_ARG;
    p->N = N;
    p->prec = prec;
    p->a = a;
    p->b = b;
    p->c = c;
    p->d = d;
    p->s = 1.0;
    p->k = lct_const(N, a, b, c, d);
    autotune_on_plan(N, (int)prec);
    *out = p;
    return LCT_OK;
}

int lct_plan_create_scaled(lct_plan *out, int64_t N, double a, double b, double c, double d, double s,
                           lct_precision prec)
{
    if (out == nullptr)
        return LCT_ERR_ARG;
    *out = nullptr;
    if (!isfinite(s) || !(s > 0.0))
        return LCT_ERR_ARG;
    lct_plan p = nullptr;
    int rc = lct_plan_create_ex(&p, N, a, b, c, d, prec);
    if (rc)
        return rc;
    const LctConst k = lct_const_scaled(N, a, b, c, d, s);
    if (!lct_const_finite(k)) {
        delete p;
        return LCT_ERR_ARG;
    }
    p->s = s;
    p->k = k;
    *out = p;
    return LCT_OK;
}

int lct_plan_create(lct_plan *out, int64_t N, double a, double b, double c, double d)
{
    return lct_plan_create_ex(out, N, a, b, c, d, LCT_FP32);
}

void lct_plan_destroy(lct_plan p) { delete p; }

int lct_exec(lct_plan p, const void *in, void *out, int64_t batch, hipStream_t stream)
{
    if (!p)
        return LCT_ERR_ARG;
    return lct_run(p->N, p->prec == LCT_FP64, p->prec == LCT_FP32_SPLITBF16, nullptr, &p->k, 0, in, out, batch, stream);
}

int lct_exec_adjoint(lct_plan p, const void *g, void *out, int64_t batch, hipStream_t stream)
{
    if (!p)
        return LCT_ERR_ARG;
    if (p->b == 0.0)
        return LCT_ERR_UNSUPPORTED;
    return lct_run(p->N, p->prec == LCT_FP64, p->prec == LCT_FP32_SPLITBF16, nullptr, &p->k, 1, g, out, batch, stream);
}

int lct_exec_many(int64_t N, lct_precision prec, const double *M4, const void *in, void *out, int64_t batch,
                  hipStream_t stream)
{
    if (prec != LCT_FP32 && prec != LCT_FP64 && prec != LCT_FP32_SPLITBF16)
        return LCT_ERR_ARG;
    if (batch > 0 && (M4 == nullptr || ((uintptr_t)M4) % 8))
        return LCT_ERR_ARG;
    return lct_run(N, prec == LCT_FP64, prec == LCT_FP32_SPLITBF16, M4, nullptr, 0, in, out, batch, stream);
}

int lct_exec_many_adjoint(int64_t N, lct_precision prec, const double *M4, const void *g, void *out, int64_t batch,
                          hipStream_t stream)
{
    if (prec != LCT_FP32 && prec != LCT_FP64 && prec != LCT_FP32_SPLITBF16)
        return LCT_ERR_ARG;
    if (batch > 0 && (M4 == nullptr || ((uintptr_t)M4) % 8))
        return LCT_ERR_ARG;
    return lct_run(N, prec == LCT_FP64, prec == LCT_FP32_SPLITBF16, M4, nullptr, 1, g, out, batch, stream);
}

int lct_param_grad_many(int64_t N, lct_precision prec, const double *M4, const void *f, const void *g,
                        double *grad4, int64_t batch, hipStream_t stream)
{
    if (prec == LCT_FP32_SPLITBF16)
        return LCT_ERR_UNSUPPORTED;
    if (prec != LCT_FP32 && prec != LCT_FP64)
        return LCT_ERR_ARG;
    if (batch < 0)
        return LCT_ERR_ARG;
    if (!smooth235(N))
        return LCT_ERR_UNSUPPORTED_N;
    if (batch == 0)
        return LCT_OK;
    const bool fp64 = prec == LCT_FP64;
    int rc;
    if ((rc = check_ptr(f, fp64)) || (rc = check_ptr(g, fp64)))
        return rc;
    if (M4 == nullptr || ((uintptr_t)M4) % 8 || grad4 == nullptr || ((uintptr_t)grad4) % 8)
        return LCT_ERR_ARG;
    if (N > lct_max_single_pass(prec))
        return LCT_ERR_UNSUPPORTED;
    const Tiling tl = default_tiling(N, fp64, false, 0);
    if (!tl.ok)
        return LCT_ERR_UNSUPPORTED;
    LctArgs a{};
    a.N = (int)N;
    a.T = tl.T;
    a.S = tl.S;
    a.mode = 0;
    a.batch = batch;
    a.M4 = M4;
    a.nc = n_const_host(N);
    a.sc = tl.sc;
    int64_t nb = (batch + tl.S - 1) / tl.S;
    if (nb > INT32_MAX)
        return LCT_ERR_ARG;
    return hip_status(launch_pgrad(fp64, tl.E, f, g, grad4, a, (int)nb, tl.block, tl.lds, stream));
}

int frft_exec(lct_plan p, double z_re, double z_im, const void *in, void *out, int64_t batch, hipStream_t stream)
{
    if (!p)
        return LCT_ERR_ARG;
    if (p->prec == LCT_FP32_SPLITBF16)
        return LCT_ERR_UNSUPPORTED; // the fractional transform has no matrix-core variant
    if (p->s != 1.0)
        return LCT_ERR_UNSUPPORTED; // the same-grid fractional transform is defined on x_k only
    if (int rc = validate_z(z_re, z_im))
        return rc;
    FrConst k = fr_const(p->N, z_re, z_im);
    return frft_run(p->N, p->prec == LCT_FP64, nullptr, &k, in, out, batch, nullptr, 0, stream);
}

int frft_exec_ws(lct_plan p, double z_re, double z_im, const void *in, void *out, int64_t batch, void *ws,
                 size_t ws_bytes, hipStream_t stream)
{
    if (!p)
        return LCT_ERR_ARG;
    if (p->prec == LCT_FP32_SPLITBF16)
        return LCT_ERR_UNSUPPORTED; // the fractional transform has no matrix-core variant
    if (p->s != 1.0)
        return LCT_ERR_UNSUPPORTED; // the same-grid fractional transform is defined on x_k only
    if (int rc = validate_z(z_re, z_im))
        return rc;
    FrConst k = fr_const(p->N, z_re, z_im);
    return frft_run(p->N, p->prec == LCT_FP64, nullptr, &k, in, out, batch, ws, ws_bytes, stream);
}

int frft_exec_noalloc(lct_plan p, double z_re, double z_im, const void *in, void *out, int64_t batch,
                      hipStream_t stream)
{
    if (!p)
        return LCT_ERR_ARG;
    if (p->prec == LCT_FP32_SPLITBF16)
        return LCT_ERR_UNSUPPORTED;
    if (p->s != 1.0)
        return LCT_ERR_UNSUPPORTED;
    if (int rc = validate_z(z_re, z_im))
        return rc;
    if (batch < 0)
        return LCT_ERR_ARG;
    const size_t need = frft_ws_bytes(p->N, p->prec == LCT_FP64, batch);
    if (need > LCT_NOALLOC_SCRATCH_BYTES)
        return LCT_ERR_WORKSPACE;
    if (batch == 0)
        return LCT_OK;
    void *ws = nullptr;
    if (int rc = scratch_of_current_device(&ws))
        return rc;
    FrConst k = fr_const(p->N, z_re, z_im);
    return frft_run(p->N, p->prec == LCT_FP64, nullptr, &k, in, out, batch, ws, need, stream);
}

size_t lct_oversampled_workspace_size(int64_t N, int P, lct_precision prec, int64_t batch)
{
    if (!smooth235(N) || P < 1 || batch < 0 || (prec != LCT_FP32 && prec != LCT_FP64))
        return 0;
    return (size_t)batch * (size_t)P * (size_t)N * (prec == LCT_FP64 ? 16 : 8);
}

int lct_exec_oversampled(lct_plan p, int P, const void *in, void *out, int64_t batch, void *ws, size_t ws_bytes,
                         hipStream_t stream)
{
    if (!p || P < 1 || batch < 0)
        return LCT_ERR_ARG;
    if (p->prec == LCT_FP32_SPLITBF16 || p->s != 1.0)
        return LCT_ERR_UNSUPPORTED;
    // no aliasing to remove: the diagonal (b = 0), or the plain grid
    if (P == 1 || p->b == 0.0)
        return lct_exec(p, in, out, batch, stream);
    const int64_t N = p->N, M = (int64_t)P * N;
    if (((int64_t)(P - 1) * N) % 2 != 0)
        return LCT_ERR_ARG; // the y_j would fall between the fine output nodes
    const bool fp64 = p->prec == LCT_FP64;
    if (!smooth235(M))
        return LCT_ERR_UNSUPPORTED_N;
    if (M > single_pass_limit(fp64))
        return LCT_ERR_UNSUPPORTED;
    for (int q : {2, 3, 5})
        if (P % q == 0 && N % q != 0)
            return LCT_ERR_UNSUPPORTED; // the two DFTs share one thread layout
    if (batch == 0)
        return LCT_OK;
    int rc;
    if ((rc = check_ptr(in, fp64)) || (rc = check_ptr(out, fp64)))
        return rc;
    const size_t need = (size_t)batch * (size_t)M * (fp64 ? 16 : 8);
    if (ws == nullptr || ws_bytes < need || ((uintptr_t)ws) % 16)
        return LCT_ERR_WORKSPACE;
    if (batch > INT32_MAX)
        return LCT_ERR_ARG;
    // values per thread: E divides N (and so P N), schedules with radices
    // dividing E exist for both lengths, at most 1024 threads
    InterpArgs a{};
    // (the fused kernel's width first where it has an instantiation; otherwise
    // FP64 tries 8 first: at E = 16 the interpolation kernel spills)
    int E = 0;
    static const int widths32[] = {16, 20, 24, 12, 10, 8, 15, 6, 5, 4, 3, 2};
    static const int widths64[] = {8, 16, 12, 10, 20, 24, 6, 15, 5, 4, 3, 2};
    const int *widths = fp64 ? widths64 : widths32;
    const int fw = oversampled_fused_width(fp64, (int)N, (int)M);
    for (int w = fw > 0 ? -1 : 0; w < 12; ++w) {
        const int cand = w < 0 ? fw : widths[w];
        if (N % cand || M / cand > 1024 || !interp_width_ok(cand))
            continue;
        const Sched s1 = greedy_sched(N, cand, 16, false), s2 = greedy_sched(M, cand, 16, false);
        if (s1.nst < 0 || s2.nst < 0)
            continue;
        E = cand;
        a.sc1 = s1;
        a.sc2 = s2;
        break;
    }
    if (E == 0)
        return LCT_ERR_UNSUPPORTED;
    a.N = (int)N;
    a.P = P;
    a.T = (int)(M / E);
    a.T1 = (int)(N / E);
    a.batch = batch;
    const size_t lds = (size_t)lds_elems((int)M) * (fp64 ? 16 : 8);
    if (lds > LDS_BYTES)
        return LCT_ERR_UNSUPPORTED;
    // the fine grid is the scaled grid s x'_m of M points, s = 1 / sqrt(P):
    // step h / P over the same span; its outputs 4 b x'_m / (pi s) hold the
    // Algorithm's y_j at m = j + (P - 1) N / 2
    const LctConst k = lct_const_scaled(M, p->a, p->b, p->c, p->d, 1.0 / sqrt((double)P));
    if (!lct_const_finite(k))
        return LCT_ERR_ARG;
    const int off = (int)((P - 1) * N / 2);
    a.k = k;
    // one kernel for the interpolation, the fine transform and the window where
    // an instantiation exists (the fine samples stay on chip)
    const hipError_t fe = launch_oversampled_fused(fp64, E, in, out, a, lds, stream);
    if (fe != hipErrorNotSupported)
        return hip_status(fe);
    if ((rc = hip_status(launch_interp(fp64, E, in, ws, a, lds, stream))))
        return rc;
    // the fine transform stores only its middle block straight to out where a
    // windowed instantiation exists; otherwise in full, then the window is copied
    rc = lct_launch_window(M, fp64, &k, ws, out, batch, off, (int)N, stream);
    if (rc != LCT_ERR_UNSUPPORTED)
        return rc;
    if ((rc = lct_run(M, fp64, false, nullptr, &k, 0, ws, ws, batch, stream)))
        return rc;
    return hip_status(launch_window(fp64, ws, out, (int)N, (int)M, off, batch, stream));
}

int lct_complex_exec(int64_t N, lct_precision prec, double a_re, double a_im, double b_re, double b_im, double d_re,
                     double d_im, const void *in, void *out, int64_t batch, hipStream_t stream)
{
    if (prec == LCT_FP32_SPLITBF16)
        return LCT_ERR_UNSUPPORTED;
    if (prec != LCT_FP32 && prec != LCT_FP64)
        return LCT_ERR_ARG;
    for (double v : {a_re, a_im, b_re, b_im, d_re, d_im})
        if (!isfinite(v))
            return LCT_ERR_ARG;
    if (b_re == 0.0 && b_im == 0.0)
        return LCT_ERR_UNSUPPORTED; // the b = 0 diagonal samples f at d y_j, off the grid for complex d
    if (!smooth235(N))
        return LCT_ERR_UNSUPPORTED_N;
    const bool fp64 = prec == LCT_FP64;
    if (N > single_pass_limit(fp64))
        return LCT_ERR_UNSUPPORTED;
    CxArgs a{};
    if (int rc = cx_const(N, a_re, a_im, b_re, b_im, d_re, d_im, &a.k))
        return rc;
    if (batch < 0)
        return LCT_ERR_ARG;
    if (batch == 0)
        return LCT_OK;
    int rc;
    if ((rc = check_ptr(in, fp64)) || (rc = check_ptr(out, fp64)))
        return rc;
    const Tiling tl = default_tiling(N, fp64, false, 0);
    if (!tl.ok)
        return LCT_ERR_UNSUPPORTED;
    a.N = (int)N;
    a.T = tl.T;
    a.S = tl.S;
    a.batch = batch;
    a.sc = tl.sc;
    const int64_t nb = (batch + tl.S - 1) / tl.S;
    if (nb > INT32_MAX)
        return LCT_ERR_ARG;
    return hip_status(launch_cx(fp64, tl.E, in, out, a, (int)nb, tl.block, tl.lds, stream));
}

int lct_complex_nodes(int64_t N, double b_re, double b_im, double *y)
{
    if (N < 1 || y == nullptr || (b_re == 0.0 && b_im == 0.0) || !isfinite(b_re) || !isfinite(b_im))
        return LCT_ERR_ARG;
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double s = 4.0L / pi * (pi / (2.0L * sqrtl(2.0L * (long double)N)));
    for (int64_t j = 0; j < N; ++j) {
        const long double x = s * (long double)(2 * j - N + 1);
        y[2 * j] = (double)(x * (long double)b_re);
        y[2 * j + 1] = (double)(x * (long double)b_im);
    }
    return LCT_OK;
}

int lct_same_grid_exec(int64_t N, lct_precision prec, double a_re, double a_im, double b_re, double b_im,
                       double d_re, double d_im, const void *in, void *out, int64_t batch, void *ws,
                       size_t ws_bytes, hipStream_t stream)
{
    if (prec == LCT_FP32_SPLITBF16)
        return LCT_ERR_UNSUPPORTED;
    if (prec != LCT_FP32 && prec != LCT_FP64)
        return LCT_ERR_ARG;
    for (double v : {a_re, a_im, b_re, b_im, d_re, d_im})
        if (!isfinite(v))
            return LCT_ERR_ARG;
    if (b_re == 0.0 && b_im == 0.0)
        return LCT_ERR_UNSUPPORTED; // b = 0 samples f at d y_j, off the grid
    if (!smooth235(N))
        return LCT_ERR_UNSUPPORTED_N;
    FrConst k;
    const int rc = same_grid_const(N, a_re, a_im, b_re, b_im, d_re, d_im, &k);
    if (rc)
        return rc;
    return frft_run(N, prec == LCT_FP64, nullptr, &k, in, out, batch, ws, ws_bytes, stream);
}

size_t frft_workspace_size(int64_t N, lct_precision prec, int64_t batch)
{
    if (!smooth235(N) || batch < 0 || (prec != LCT_FP32 && prec != LCT_FP64))
        return 0;
    return frft_ws_bytes(N, prec == LCT_FP64, batch);
}

int frft_exec_many(int64_t N, lct_precision prec, const double *Z2, const void *in, void *out, int64_t batch,
                   hipStream_t stream)
{
    if (prec == LCT_FP32_SPLITBF16)
        return LCT_ERR_UNSUPPORTED;
    if (prec != LCT_FP32 && prec != LCT_FP64)
        return LCT_ERR_ARG;
    if (batch > 0 && (Z2 == nullptr || ((uintptr_t)Z2) % 8))
        return LCT_ERR_ARG;
    return frft_run(N, prec == LCT_FP64, Z2, nullptr, in, out, batch, nullptr, 0, stream);
}

int frft_exec_many_ws(int64_t N, lct_precision prec, const double *Z2, const void *in, void *out, int64_t batch,
                      void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (prec == LCT_FP32_SPLITBF16)
        return LCT_ERR_UNSUPPORTED;
    if (prec != LCT_FP32 && prec != LCT_FP64)
        return LCT_ERR_ARG;
    if (batch > 0 && (Z2 == nullptr || ((uintptr_t)Z2) % 8))
        return LCT_ERR_ARG;
    return frft_run(N, prec == LCT_FP64, Z2, nullptr, in, out, batch, ws, ws_bytes, stream);
}

int lct_nodes(int64_t N, double b, double d, double *x, double *y)
{
    if (N < 1 || (b == 0.0 && d == 0.0))
        return LCT_ERR_ARG;
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double h = pi / sqrtl(2.0L * (long double)N);
    for (int64_t k = 0; k < N; ++k) {
        long double xk = h * (long double)(2 * k - N + 1) / 2.0L;
        if (x)
            x[k] = (double)xk;
        if (y)
            y[k] = (double)(b != 0.0 ? 4.0L * (long double)b * xk / pi : xk / (long double)d);
    }
    return LCT_OK;
}

int lct_nodes_scaled(int64_t N, double b, double d, double s, double *x, double *y)
{
    if (N < 1 || (b == 0.0 && d == 0.0) || !isfinite(s) || !(s > 0.0))
        return LCT_ERR_ARG;
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double h = pi / sqrtl(2.0L * (long double)N), S = s;
    for (int64_t k = 0; k < N; ++k) {
        long double xk = h * (long double)(2 * k - N + 1) / 2.0L;
        if (x)
            x[k] = (double)(S * xk);
        if (y)
            y[k] = (double)(b != 0.0 ? 4.0L * (long double)b * xk / (pi * S) : S * xk / (long double)d);
    }
    return LCT_OK;
}

const char *lct_strerror(int code)
{
    switch (code) {
    case LCT_OK:
        return "success";
    case LCT_ERR_ARG:
        return "invalid argument (null or misaligned pointer, negative batch, bad enum)";
    case LCT_ERR_NOT_UNIMODULAR:
        return "matrix (a b; c d) is not unimodular: |ad - bc - 1| > 1e-10 max(1, |ad|, |bc|)";
    case LCT_ERR_UNSUPPORTED_N:
        return "N must be 2^p 3^q 5^r with 1 <= N <= 2^24";
    case LCT_ERR_DOMAIN:
        return "fractional order outside the closed unit disc";
    case LCT_ERR_WORKSPACE:
        return "workspace missing or too small";
    case LCT_ERR_HIP:
        return "HIP runtime error";
    case LCT_ERR_UNSUPPORTED:
        return "request not supported by this build";
    default:
        return "unknown error code";
    }
}

} // extern "C"
