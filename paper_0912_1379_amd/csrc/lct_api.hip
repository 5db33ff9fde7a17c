// lct_api.hip - host side of the C ABI declared in include/lct.h: argument
// validation, plan constants, size/tiling selection and kernel dispatch.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include <new>

#include "../../include/lct.h"
#include "lct_kernels.hpp"

using namespace lctk;

struct lct_plan_s {
    int64_t N;
    int prec;
    double a, b, c, d;
    LctConst k;
};

namespace {

constexpr int64_t MAX_N = int64_t(1) << 24;
constexpr size_t LDS_BYTES = 160 * 1024;

bool smooth235(int64_t N)
{
    if (N < 1 || N > MAX_N)
        return false;
    for (int p : {2, 3, 5})
        while (N % p == 0)
            N /= p;
    return N == 1;
}

// Elements per thread: the first E of the list for the size's prime set that
// divides N and keeps the thread count per signal within a work-group.
int choose_E(int64_t N, bool fp64, bool frft)
{
    int64_t m = N;
    bool p2 = false, p3 = false, p5 = false;
    while (m % 2 == 0) { m /= 2; p2 = true; }
    while (m % 3 == 0) { m /= 3; p3 = true; }
    while (m % 5 == 0) { m /= 5; p5 = true; }
    static const int l2[] = {16, 8, 4, 2, 0};
    static const int l3[] = {27, 9, 3, 0};
    static const int l5[] = {25, 5, 0};
    static const int l23[] = {24, 12, 6, 18, 0};
    static const int l25[] = {20, 10, 0};
    static const int l35[] = {15, 0};
    static const int l235[] = {30, 0};
    static const int l1[] = {1, 0};
    static const int l2_64[] = {16, 8, 4, 2, 0};
    static const int l23_64[] = {12, 6, 24, 18, 0};
    static const int l25_64[] = {10, 20, 0};
    static const int l2_fr[] = {16, 8, 4, 2, 0};
    static const int l2_fr64[] = {8, 16, 4, 2, 0};
    const int *lst;
    if (p2 && p3 && p5) lst = l235;
    else if (p2 && p3) lst = fp64 ? l23_64 : l23;
    else if (p2 && p5) lst = fp64 ? l25_64 : l25;
    else if (p3 && p5) lst = l35;
    else if (p2) lst = frft ? (fp64 ? l2_fr64 : l2_fr) : (fp64 ? l2_64 : l2);
    else if (p3) lst = l3;
    else if (p5) lst = l5;
    else lst = l1;
    for (int i = 0; lst[i]; ++i) {
        int E = lst[i];
        if (N % E == 0 && N / E <= max_block(fp64, E))
            return E;
    }
    return 0;
}

Sched make_sched(int64_t N, int E)
{
    Sched s{};
    s.nst = 0;
    int64_t rem = N;
    const int cand[6] = {16, 8, 5, 4, 3, 2};
    while (rem > 1 && s.nst < 24) {
        bool ok = false;
        for (int c : cand) {
            if (E % c == 0 && rem % c == 0) {
                s.rad[s.nst++] = c;
                rem /= c;
                ok = true;
                break;
            }
        }
        if (!ok)
            break;
    }
    if (rem != 1)
        s.nst = -1;
    return s;
}

struct Tiling {
    int E = 0, T = 0, S = 0, block = 0;
    size_t lds = 0;
    Sched sc{};
    bool ok = false;
};

// Length Nfft DFT held in LDS; `extra` bytes per signal slot after the FFT area.
Tiling make_tiling(int64_t Nfft, bool fp64, bool frft, size_t extra)
{
    Tiling t;
    t.E = choose_E(Nfft, fp64, frft);
    if (t.E == 0)
        return t;
    t.T = (int)(Nfft / t.E);
    t.sc = make_sched(Nfft, t.E);
    if (t.sc.nst < 0)
        return t;
    const size_t elem = fp64 ? 16 : 8;
    const size_t per = (size_t)lds_elems((int)Nfft) * elem;
    int S = t.T >= 256 ? 1 : 256 / t.T;
    if (S < 1)
        S = 1;
    while (S > 1 && S * (per + extra) > LDS_BYTES)
        --S;
    if (per + extra > LDS_BYTES)
        return t;
    t.S = S;
    t.block = S * t.T;
    t.lds = S * per + S * extra;
    t.ok = t.block <= max_block(fp64, t.E);
    return t;
}

int hip_status(hipError_t e);

// Two-pass (four-step) plan for N beyond one work-group: N = N1 N2 with N1 the
// largest divisor <= sqrt(N) whose tiles fit; C columns per pass-1 group and
// RR rows per pass-2 group, as many as keep >= 128-byte row segments and fit
// LDS and the launch bound.
struct FsTiling {
    int N1 = 0, N2 = 0, E1 = 0, E2 = 0, T1 = 0, T2 = 0, C = 0, RR = 0, bs1 = 0, bs2 = 0;
    size_t lds1 = 0, lds2 = 0;
    Sched sc1{}, sc2{};
    bool ok = false;
};

int pick_group(int Nsub, int T, int E, int other, bool fp64)
{
    const size_t elem = fp64 ? 16 : 8;
    const size_t per = (size_t)lds_elems(Nsub) * elem;
    const int want = fp64 ? 8 : 16;          // >= 128 B per row segment
    int cap = 256 / T > want ? 256 / T : want; // ~256 threads when T is small
    if (cap > 64)
        cap = 64;
    for (int c = cap; c >= 1; --c) {
        if (other % c)
            continue;
        if (c * T > max_block(fp64, E) || c * per > LDS_BYTES)
            continue;
        return c;
    }
    return 0;
}

FsTiling make_fs(int64_t N, bool fp64)
{
    FsTiling f;
    int64_t best = 0;
    for (int64_t d = 1; d * d <= N; ++d)
        if (N % d == 0)
            best = d;
    for (int64_t N1 = best; N1 >= 2; --N1) {
        if (N % N1)
            continue;
        const int64_t N2 = N / N1;
        if (N1 > 16384 || N2 > 16384)
            break;
        f.N1 = (int)N1;
        f.N2 = (int)N2;
        f.E1 = choose_E(N1, fp64, false);
        f.E2 = choose_E(N2, fp64, false);
        if (!f.E1 || !f.E2)
            continue;
        f.T1 = (int)(N1 / f.E1);
        f.T2 = (int)(N2 / f.E2);
        f.sc1 = make_sched(N1, f.E1);
        f.sc2 = make_sched(N2, f.E2);
        if (f.sc1.nst < 0 || f.sc2.nst < 0)
            continue;
        f.C = pick_group((int)N1, f.T1, f.E1, (int)N2, fp64);
        f.RR = pick_group((int)N2, f.T2, f.E2, (int)N1, fp64);
        if (!f.C || !f.RR)
            continue;
        const size_t elem = fp64 ? 16 : 8;
        f.bs1 = f.C * f.T1;
        f.bs2 = f.RR * f.T2;
        f.lds1 = (size_t)f.C * lds_elems((int)N1) * elem;
        f.lds2 = (size_t)f.RR * lds_elems((int)N2) * elem;
        f.ok = true;
        return f;
    }
    f.ok = false;
    return f;
}

int fs_run(int64_t N, bool fp64, const double *M4, const LctConst *k, int mode, const void *in, void *out,
           int64_t batch, hipStream_t s)
{
    if (in == out)
        return LCT_ERR_ARG; // pass 1 reads columns of `in` while writing rows of `out`
    FsTiling f = make_fs(N, fp64);
    if (!f.ok)
        return LCT_ERR_UNSUPPORTED;
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
    hipError_t e = launch_fs1(fp64, f.E1, in, out, a, (int)nb1, f.bs1, f.lds1, s);
    if (e != hipSuccess)
        return LCT_ERR_HIP;
    return hip_status(launch_fs2(fp64, f.E2, out, a, (int)nb2, f.bs2, f.lds2, s));
}

int check_ptr(const void *p, bool fp64)
{
    if (p == nullptr)
        return LCT_ERR_ARG;
    if (((uintptr_t)p) % (fp64 ? 16 : 8) != 0)
        return LCT_ERR_ARG;
    return LCT_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? LCT_OK : LCT_ERR_HIP; }

int validate_M(double a, double b, double c, double d)
{
    if (!isfinite(a) || !isfinite(b) || !isfinite(c) || !isfinite(d))
        return LCT_ERR_ARG;
    double ad = a * d, bc = b * c;
    double tol = 1e-10 * fmax(1.0, fmax(fabs(ad), fabs(bc)));
    if (fabs(ad - bc - 1.0) > tol)
        return LCT_ERR_NOT_UNIMODULAR;
    return LCT_OK;
}

int lct_run(int64_t N, bool fp64, const double *M4, const LctConst *k, int mode, const void *in, void *out,
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
    if (N > lct_max_single_pass(fp64 ? LCT_FP64 : LCT_FP32))
        return fs_run(N, fp64, M4, k, mode, in, out, batch, s);
    Tiling tl = make_tiling(N, fp64, false, 0);
    if (!tl.ok)
        return LCT_ERR_UNSUPPORTED;
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
    int64_t nb = (batch + tl.S - 1) / tl.S;
    if (nb > INT32_MAX)
        return LCT_ERR_ARG;
    return hip_status(launch_lct(fp64, tl.E, in, out, a, (int)nb, tl.block, tl.lds, s));
}

size_t frft_ws_bytes(int64_t N, bool fp64, int64_t batch)
{
    if (2 * N <= lct_max_single_pass(fp64 ? LCT_FP64 : LCT_FP32))
        return 0;
    return (size_t)batch * 2 * (size_t)(2 * N) * (fp64 ? 16 : 8);
}

int frft_large(int64_t N, bool fp64, const double *Z2, const FrConst *k, const void *in, void *out, int64_t batch,
               void *ws, hipStream_t s)
{
    FsTiling f = make_fs(2 * N, fp64);
    if (!f.ok)
        return LCT_ERR_UNSUPPORTED;
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
    if (2 * nb1 > INT32_MAX || 2 * nb2 > INT32_MAX || batch > INT32_MAX)
        return LCT_ERR_ARG;
    hipError_t e;
    if ((e = launch_frl1(fp64, f.E1, in, ws, a, (int)(2 * nb1), f.bs1, f.lds1, s)) != hipSuccess ||
        (e = launch_frl2(fp64, f.E2, ws, a, (int)nb2, f.bs2, f.lds2, s)) != hipSuccess ||
        (e = launch_frl3(fp64, f.E1, ws, out, a, (int)nb1, f.bs1, f.lds1, s)) != hipSuccess)
        return LCT_ERR_HIP;
    if (Z2 != nullptr || (k && k->special))
        return hip_status(launch_fr_special(fp64, in, out, a, s));
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
    if (2 * N > lct_max_single_pass(fp64 ? LCT_FP64 : LCT_FP32)) {
        const size_t need = frft_ws_bytes(N, fp64, batch);
        if (ws == nullptr || ws_bytes < need || ((uintptr_t)ws) % 16)
            return LCT_ERR_WORKSPACE;
        return frft_large(N, fp64, Z2, k, in, out, batch, ws, s);
    }
    Tiling tl = make_tiling(2 * N, fp64, true, 0);
    if (!tl.ok)
        return LCT_ERR_UNSUPPORTED;
    FrArgs a{};
    a.N = (int)N;
    a.T = tl.T;
    a.S = tl.S;
    a.batch = batch;
    a.Z2 = Z2;
    if (k)
        a.k = *k;
    a.sc = tl.sc;
    int64_t nb = (batch + tl.S - 1) / tl.S;
    if (nb > INT32_MAX)
        return LCT_ERR_ARG;
    return hip_status(launch_frft(fp64, tl.E, in, out, a, (int)nb, tl.block, tl.lds, s));
}

} // namespace

extern "C" {

int64_t lct_max_single_pass(lct_precision prec)
{
    // largest 2^p 3^q 5^r whose padded LDS image fits 160 KiB with <= 1024 threads
    return prec == LCT_FP64 ? 8192 : 16384;
}

int lct_plan_create_ex(lct_plan *out, int64_t N, double a, double b, double c, double d, lct_precision prec)
{
    if (out == nullptr)
        return LCT_ERR_ARG;
    *out = nullptr;
    if (prec != LCT_FP32 && prec != LCT_FP64)
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
    p->k = lct_const(N, a, b, c, d);
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
    return lct_run(p->N, p->prec == LCT_FP64, nullptr, &p->k, 0, in, out, batch, stream);
}

int lct_exec_adjoint(lct_plan p, const void *g, void *out, int64_t batch, hipStream_t stream)
{
    if (!p)
        return LCT_ERR_ARG;
    if (p->b == 0.0)
        return LCT_ERR_UNSUPPORTED;
    return lct_run(p->N, p->prec == LCT_FP64, nullptr, &p->k, 1, g, out, batch, stream);
}

int lct_exec_many(int64_t N, lct_precision prec, const double *M4, const void *in, void *out, int64_t batch,
                  hipStream_t stream)
{
    if (prec != LCT_FP32 && prec != LCT_FP64)
        return LCT_ERR_ARG;
    if (batch > 0 && (M4 == nullptr || ((uintptr_t)M4) % 8))
        return LCT_ERR_ARG;
    return lct_run(N, prec == LCT_FP64, M4, nullptr, 0, in, out, batch, stream);
}

int lct_exec_many_adjoint(int64_t N, lct_precision prec, const double *M4, const void *g, void *out, int64_t batch,
                          hipStream_t stream)
{
    if (prec != LCT_FP32 && prec != LCT_FP64)
        return LCT_ERR_ARG;
    if (batch > 0 && (M4 == nullptr || ((uintptr_t)M4) % 8))
        return LCT_ERR_ARG;
    return lct_run(N, prec == LCT_FP64, M4, nullptr, 1, g, out, batch, stream);
}

int lct_param_grad_many(int64_t N, lct_precision prec, const double *M4, const void *f, const void *g,
                        double *grad4, int64_t batch, hipStream_t stream)
{
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
    Tiling tl = make_tiling(N, fp64, false, 3 * sizeof(double));
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
    if (!isfinite(z_re) || !isfinite(z_im))
        return LCT_ERR_ARG;
    if (hypot(z_re, z_im) > 1.0 + 1e-12)
        return LCT_ERR_DOMAIN;
    FrConst k = fr_const(p->N, z_re, z_im);
    return frft_run(p->N, p->prec == LCT_FP64, nullptr, &k, in, out, batch, nullptr, 0, stream);
}

int frft_exec_ws(lct_plan p, double z_re, double z_im, const void *in, void *out, int64_t batch, void *ws,
                 size_t ws_bytes, hipStream_t stream)
{
    if (!p)
        return LCT_ERR_ARG;
    if (!isfinite(z_re) || !isfinite(z_im))
        return LCT_ERR_ARG;
    if (hypot(z_re, z_im) > 1.0 + 1e-12)
        return LCT_ERR_DOMAIN;
    FrConst k = fr_const(p->N, z_re, z_im);
    return frft_run(p->N, p->prec == LCT_FP64, nullptr, &k, in, out, batch, ws, ws_bytes, stream);
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
    if (prec != LCT_FP32 && prec != LCT_FP64)
        return LCT_ERR_ARG;
    if (batch > 0 && (Z2 == nullptr || ((uintptr_t)Z2) % 8))
        return LCT_ERR_ARG;
    return frft_run(N, prec == LCT_FP64, Z2, nullptr, in, out, batch, nullptr, 0, stream);
}

int frft_exec_many_ws(int64_t N, lct_precision prec, const double *Z2, const void *in, void *out, int64_t batch,
                      void *ws, size_t ws_bytes, hipStream_t stream)
{
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
