// xft.hip - the exact-node discrete fractional transform of §2 (eq. tmat):
// plan (zeros of H_N and the orthonormal vectors of eq. ortvec, computed on
// the host and kept on the device) and the two matrix-core passes.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <thread>
#include <vector>

#include "../../include/lct.h"
#include "lct_kernels.hpp"
#include "xft_impl.hpp"

using namespace lctk;

struct xft_plan_s {
    int64_t N;
    int prec;
    void *U;  // N x N, U[n][k] = (u_k)_n, in the plan's precision (device)
    void *Ut; // its transpose (device)
    // split-BF16 plans: U and U^T as hi + lo BF16 parts, rows padded to ldb
    void *Uh, *Ul, *Uth, *Utl;
    int ldb;
};

namespace {

constexpr int64_t XFT_MAX_N = 16384;

// Runs body(lo, hi) over [0, n) split across up to 16 host threads (the
// per-zero and per-vector work below is independent).
template <typename F>
void parallel_ranges(int64_t n, F body)
{
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::min<int64_t>(std::max<unsigned>(hw, 1u), 16);
    nt = std::min<int64_t>(nt, std::max<int64_t>(1, n / 4));
    if (nt <= 1) {
        body(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    for (int64_t i = 0; i < nt; ++i)
        th.emplace_back(body, n * i / nt, n * (i + 1) / nt);
    for (auto &t : th)
        t.join();
}

// One implicit symmetric QR step with a Wilkinson shift on the unreduced
// block [lo, hi] of a symmetric tridiagonal matrix (diagonal al, off-diagonal
// be, be[i] coupling i and i + 1), as in Golub & Van Loan, "Matrix
// Computations", the implicit symmetric QR step (Algorithm 8.3.2): the shift
// mu is the eigenvalue of the trailing 2 x 2 block nearer its last diagonal
// entry; a plane rotation in (lo, lo + 1) taken from the first column of
// T - mu I creates a bulge below the subdiagonal, and rotations in
// (k, k + 1), k = lo + 1 .. hi - 1, chase it off the bottom.  Each rotation
// is applied as a similarity T <- G^T T G to the 2 x 2 diagonal block it
// touches and to its two neighbouring couplings.
void qr_step_wilkinson(double *al, double *be, int64_t lo, int64_t hi)
{
    const double half_gap = 0.5 * (al[hi - 1] - al[hi]);
    const double last = be[hi - 1];
    const double mu = al[hi] - last * last / (half_gap + copysign(hypot(half_gap, last), half_gap));
    double x = al[lo] - mu; // entry to keep
    double z = be[lo];      // entry to annihilate
    for (int64_t k = lo; k < hi; ++k) {
        // rotation [c s; -s c] with [c s; -s c]^T (x, z) = (r, 0)
        double c = 1.0, s = 0.0;
        if (z != 0.0) {
            const double r = hypot(x, z);
            c = x / r;
            s = -z / r;
            if (k > lo)
                be[k - 1] = r; // the coupling that held the bulge's partner
        }
        const double p = al[k], q = al[k + 1], o = be[k];
        const double cc = c * c, ss = s * s, cs = c * s;
        al[k] = cc * p - 2.0 * cs * o + ss * q;
        al[k + 1] = ss * p + 2.0 * cs * o + cc * q;
        be[k] = cs * (p - q) + (cc - ss) * o;
        if (k + 1 < hi) {
            // the rotation spills into the coupling (k, k + 2): the next bulge
            const double nxt = be[k + 1];
            z = -s * nxt;
            be[k + 1] = c * nxt;
            x = be[k];
        }
    }
}

// Eigenvalues of the symmetric tridiagonal matrix H of §2 (zero diagonal,
// off-diagonal sqrt(i / 2), i = 1 .. N-1), i.e. the zeros of H_N, by the
// symmetric QR algorithm (Golub & Van Loan, Algorithm 8.3.3): couplings
// below eps (|al_i| + |al_{i+1}|) are set to zero, and implicit Wilkinson
// steps run on the lowest unreduced block until the matrix is diagonal;
// O(N^2) for the eigenvalues alone.  Returns them ascending in x.
void tridiag_zeros(int64_t N, std::vector<double> &x)
{
    std::vector<double> al((size_t)N, 0.0), be((size_t)(N > 1 ? N - 1 : 1), 0.0);
    for (int64_t i = 0; i + 1 < N; ++i)
        be[(size_t)i] = sqrt((double)(i + 1) / 2.0);
    const double eps = 0x1p-52;
    int64_t hi = N - 1;
    int64_t guard = 64 * (N + 1); // the shifted iteration needs about two steps per eigenvalue
    while (hi > 0 && guard-- > 0) {
        for (int64_t i = 0; i < hi; ++i)
            if (fabs(be[(size_t)i]) <= eps * (fabs(al[(size_t)i]) + fabs(al[(size_t)i + 1])))
                be[(size_t)i] = 0.0;
        while (hi > 0 && be[(size_t)hi - 1] == 0.0)
            --hi; // al[hi] has converged
        if (hi == 0)
            break;
        int64_t lo = hi - 1;
        while (lo > 0 && be[(size_t)lo - 1] != 0.0)
            --lo;
        qr_step_wilkinson(al.data(), be.data(), lo, hi);
    }
    x = al;
    std::sort(x.begin(), x.end());
}

// Newton steps on the normalised Hermite function phi_N at each zero, with
// phi_N'(x) = sqrt(2N) phi_{N-1}(x) at a zero of phi_N (from the
// derivative identity H_N' = 2N H_{N-1}); values through the three-term
// recurrence of eq. (receqg) divided by sqrt(2^n n!), rescaled against
// overflow.  The zeros are symmetric about 0: the upper half is polished and
// mirrored.
void polish_zeros(int64_t N, std::vector<double> &x)
{
    std::vector<double> a((size_t)N), b((size_t)N);
    for (int64_t n = 0; n < N; ++n) {
        a[(size_t)n] = sqrt(2.0 / (double)(n + 1));
        b[(size_t)n] = sqrt((double)n / (double)(n + 1));
    }
    parallel_ranges(N - N / 2, [&](int64_t lo, int64_t hi) {
    for (int64_t k = N / 2 + lo; k < N / 2 + hi; ++k) {
        double xk = x[(size_t)k];
        for (int it = 0; it < 3; ++it) {
            double pm = 0.0, p = 1.0; // phi_{n-1}, phi_n up to a common factor
            for (int64_t n = 0; n < N; ++n) {
                const double pn = a[(size_t)n] * xk * p - b[(size_t)n] * pm;
                pm = p;
                p = pn;
                if (fabs(p) > 0x1p400) {
                    p *= 0x1p-400;
                    pm *= 0x1p-400;
                }
            }
            // p = phi_N, pm = phi_{N-1} (same factor)
            if (pm == 0.0)
                break;
            const double dx = p / (sqrt(2.0 * (double)N) * pm);
            xk -= dx;
            if (fabs(dx) <= 1e-17 * (1.0 + fabs(xk)))
                break;
        }
        x[(size_t)k] = xk;
        x[(size_t)(N - 1 - k)] = -xk;
    }
    });
    if (N % 2 == 1)
        x[(size_t)(N / 2)] = 0.0;
}

// Ut[k][n] = (u_k)_n of eq. (ortvec), 0-based (row k of Ut is column k of U):
//   (u_k)_n = (-1)^(N+k+1) phi_n(x_k) / (sqrt(N) phi_{N-1}(x_k)),
// the normalisation being the Christoffel-Darboux sum
// sum_n phi_n(x_k)^2 = N phi_{N-1}(x_k)^2 at a zero of phi_N.  Each vector
// runs the recurrence once, keeping a running power-of-two exponent per n so
// that no earlier value is rescaled; values 2^-1200 below the last one and
// smaller underflow to zero.
void ortho_vectors_t(int64_t N, const std::vector<double> &x, double *Ut)
{
    const double down[4] = {1.0, 0x1p-400, 0x1p-800, 0.0};
    std::vector<double> a((size_t)N), b((size_t)N);
    for (int64_t n = 0; n < N; ++n) {
        a[(size_t)n] = sqrt(2.0 / (double)(n + 1));
        b[(size_t)n] = sqrt((double)n / (double)(n + 1));
    }
    const double rn = 1.0 / sqrt((double)N);
    parallel_ranges(N, [&](int64_t lo, int64_t hi) {
    std::vector<double> val((size_t)N);
    std::vector<int> ex((size_t)N);
    for (int64_t k = lo; k < hi; ++k) {
        const double xk = x[(size_t)k];
        double pm = 0.0, p = 1.0;
        int e = 0;
        val[0] = 1.0;
        ex[0] = 0;
        for (int64_t n = 0; n + 1 < N; ++n) {
            double pn = a[(size_t)n] * xk * p - b[(size_t)n] * pm;
            pm = p;
            p = pn;
            if (fabs(p) > 0x1p400) {
                p *= 0x1p-400;
                pm *= 0x1p-400;
                ++e;
            }
            val[(size_t)n + 1] = p;
            ex[(size_t)n + 1] = e;
        }
        const double last = val[(size_t)N - 1];
        const int elast = ex[(size_t)N - 1];
        const double sgn = ((N + k + 1) % 2 == 0) ? 1.0 : -1.0;
        const double scale = sgn * rn / last;
        double *row = Ut + (size_t)k * (size_t)N;
        for (int64_t n = 0; n < N; ++n) {
            const int d = elast - ex[(size_t)n]; // >= 0
            row[n] = val[(size_t)n] * down[d < 3 ? d : 3] * scale;
        }
    }
    });
}

// dst = src^T for N x N row-major matrices: 32 x 32 tiles (a tile writes 32
// rows, few enough pages for the TLB), bands of tile rows across threads.
void transpose(int64_t N, const double *src, double *dst)
{
    constexpr int64_t TB = 32;
    const int64_t nb = (N + TB - 1) / TB;
    parallel_ranges(nb, [&](int64_t lo, int64_t hi) {
        for (int64_t bi = lo; bi < hi; ++bi) {
            const int64_t i0 = bi * TB, i1 = std::min(i0 + TB, N);
            for (int64_t j0 = 0; j0 < N; j0 += TB) {
                const int64_t j1 = std::min(j0 + TB, N);
                for (int64_t i = i0; i < i1; ++i)
                    for (int64_t j = j0; j < j1; ++j)
                        dst[(size_t)j * (size_t)N + (size_t)i] = src[(size_t)i * (size_t)N + (size_t)j];
            }
        }
    });
}

int host_nodes(int64_t N, std::vector<double> &x)
{
    if (N < 1 || N > XFT_MAX_N)
        return LCT_ERR_UNSUPPORTED_N;
    if (N == 1) {
        x.assign(1, 0.0);
        return LCT_OK;
    }
    tridiag_zeros(N, x);
    polish_zeros(N, x);
    return LCT_OK;
}

template <typename R>
int upload(const double *h, int64_t N, void **dst)
{
    const size_t n2 = (size_t)N * (size_t)N;
    std::vector<R> tmp(n2);
    for (size_t i = 0; i < n2; ++i)
        tmp[i] = (R)h[i];
    if (hipMalloc(dst, n2 * sizeof(R)) != hipSuccess) {
        *dst = nullptr;
        return LCT_ERR_HIP;
    }
    if (hipMemcpy(*dst, tmp.data(), n2 * sizeof(R), hipMemcpyHostToDevice) != hipSuccess)
        return LCT_ERR_HIP;
    return LCT_OK;
}

// IEEE binary32 -> bfloat16, round to nearest even (finite inputs).
uint16_t bf16_rne(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// hi = bf16(x), lo = bf16(x - hi) of every entry of the N x N matrix M,
// rows padded with zeros to ldb; uploaded to two new device arrays.
int upload_split(const double *M, int64_t N, int ldb, void **dh, void **dl)
{
    const size_t n = (size_t)N * (size_t)ldb;
    std::vector<uint16_t> h(n, 0), l(n, 0);
    for (int64_t r = 0; r < N; ++r)
        for (int64_t c = 0; c < N; ++c) {
            const double x = M[(size_t)r * (size_t)N + (size_t)c];
            const uint16_t hb = bf16_rne((float)x);
            h[(size_t)r * ldb + (size_t)c] = hb;
            l[(size_t)r * ldb + (size_t)c] = bf16_rne((float)(x - (double)bf16_value(hb)));
        }
    *dh = *dl = nullptr;
    if (hipMalloc(dh, n * 2) != hipSuccess || hipMalloc(dl, n * 2) != hipSuccess)
        return LCT_ERR_HIP;
    if (hipMemcpy(*dh, h.data(), n * 2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(*dl, l.data(), n * 2, hipMemcpyHostToDevice) != hipSuccess)
        return LCT_ERR_HIP;
    return LCT_OK;
}

hipError_t xft_launch_sb(const xft_plan_s *p, double zr, double zi, const void *in, void *out, int64_t batch,
                         void *ws, hipStream_t s)
{
    const int N = (int)p->N;
    float *w = reinterpret_cast<float *>(ws);
    float *V = w + 2 * (size_t)((N + 1) & ~1);
    hipLaunchKernelGGL(k_xft_weights<float>, dim3((N + 255) / 256), dim3(256), 0, s, zr, zi, N, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int ncol = (N + XSB_C - 1) / XSB_C;
    const int ntiles = (int)((batch + XS - 1) / XS * ncol);
    const size_t lds = xft_sb_lds_bytes();
    if ((e = allow_lds((const void *)k_xft_gemm_sb, lds)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_xft_gemm_sb, dim3(ntiles), dim3(XTHREADS), lds, s, (const float *)in,
                       (const __bf16 *)p->Uh, (const __bf16 *)p->Ul, V, (const float *)w, N, p->ldb, batch, ncol,
                       ntiles);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_xft_gemm_sb, dim3(ntiles), dim3(XTHREADS), lds, s, (const float *)V,
                       (const __bf16 *)p->Uth, (const __bf16 *)p->Utl, (float *)out, (const float *)nullptr, N,
                       p->ldb, batch, ncol, ntiles);
    return hipGetLastError();
}

template <typename R>
hipError_t xft_launch(const xft_plan_s *p, double zr, double zi, const void *in, void *out, int64_t batch, void *ws,
                      hipStream_t s)
{
    const int N = (int)p->N;
    R *w = reinterpret_cast<R *>(ws);           // N complex weights
    R *V = w + 2 * (size_t)((N + 1) & ~1);      // batch x N complex (16-byte aligned)
    hipLaunchKernelGGL(k_xft_weights<R>, dim3((N + 255) / 256), dim3(256), 0, s, zr, zi, N, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int ncol = (N + XTile<R>::C - 1) / XTile<R>::C;
    const int64_t nsig = (batch + XS - 1) / XS;
    const int ntiles = (int)(nsig * ncol);
    const size_t lds = xft_lds_bytes((int)sizeof(R));
    if ((e = allow_lds((const void *)k_xft_gemm<R>, lds)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_xft_gemm<R>, dim3(ntiles), dim3(XTHREADS), lds, s, (const R *)in, (const R *)p->U, V,
                       (const R *)w, N, batch, ncol, ntiles);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_xft_gemm<R>, dim3(ntiles), dim3(XTHREADS), lds, s, (const R *)V, (const R *)p->Ut,
                       (R *)out, (const R *)nullptr, N, batch, ncol, ntiles);
    return hipGetLastError();
}

size_t ws_bytes_of(int64_t N, bool fp64, int64_t batch)
{
    const size_t el = fp64 ? 16 : 8; // one complex value
    return (size_t)((N + 1) & ~int64_t(1)) * el + (size_t)batch * (size_t)N * el;
}

} // namespace

extern "C" {

int xft_nodes(int64_t N, double *x)
{
    if (x == nullptr)
        return LCT_ERR_ARG;
    std::vector<double> v;
    int rc = host_nodes(N, v);
    if (rc)
        return rc;
    for (int64_t k = 0; k < N; ++k)
        x[k] = v[(size_t)k];
    return LCT_OK;
}

int xft_vectors(int64_t N, double *U)
{
    if (U == nullptr)
        return LCT_ERR_ARG;
    std::vector<double> v;
    int rc = host_nodes(N, v);
    if (rc)
        return rc;
    std::vector<double> Ut((size_t)N * (size_t)N);
    ortho_vectors_t(N, v, Ut.data());
    transpose(N, Ut.data(), U);
    return LCT_OK;
}

int xft_plan_create(xft_plan *out, int64_t N, lct_precision prec)
{
    if (out == nullptr)
        return LCT_ERR_ARG;
    *out = nullptr;
    if (prec != LCT_FP32 && prec != LCT_FP64 && prec != LCT_FP32_SPLITBF16)
        return LCT_ERR_ARG;
    std::vector<double> x;
    int rc = host_nodes(N, x);
    if (rc)
        return rc;
    std::vector<double> U((size_t)N * (size_t)N), Ut((size_t)N * (size_t)N);
    ortho_vectors_t(N, x, Ut.data());
    transpose(N, Ut.data(), U.data());
    xft_plan p = new (std::nothrow) xft_plan_s{N, (int)prec, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0};
    if (!p)
        return LCT_ERR_ARG;
    const bool fp64 = prec == LCT_FP64;
    if (prec == LCT_FP32_SPLITBF16) {
        p->ldb = (int)((N + 7) / 8 * 8);
        rc = upload_split(U.data(), N, p->ldb, &p->Uh, &p->Ul);
        if (!rc)
            rc = upload_split(Ut.data(), N, p->ldb, &p->Uth, &p->Utl);
    } else {
        rc = fp64 ? upload<double>(U.data(), N, &p->U) : upload<float>(U.data(), N, &p->U);
        if (!rc)
            rc = fp64 ? upload<double>(Ut.data(), N, &p->Ut) : upload<float>(Ut.data(), N, &p->Ut);
    }
    if (rc) {
        xft_plan_destroy(p);
        return rc;
    }
    *out = p;
    return LCT_OK;
}

void xft_plan_destroy(xft_plan p)
{
    if (!p)
        return;
    if (p->U)
        (void)hipFree(p->U);
    if (p->Ut)
        (void)hipFree(p->Ut);
    for (void *q : {p->Uh, p->Ul, p->Uth, p->Utl})
        if (q)
            (void)hipFree(q);
    delete p;
}

size_t xft_workspace_size(int64_t N, lct_precision prec, int64_t batch)
{
    if (N < 1 || N > XFT_MAX_N || batch < 0 || (prec != LCT_FP32 && prec != LCT_FP64 && prec != LCT_FP32_SPLITBF16))
        return 0;
    return ws_bytes_of(N, prec == LCT_FP64, batch);
}

int xft_exec(xft_plan p, double z_re, double z_im, const void *in, void *out, int64_t batch, void *ws,
             size_t ws_bytes, hipStream_t stream)
{
    if (!p || batch < 0)
        return LCT_ERR_ARG;
    if (!isfinite(z_re) || !isfinite(z_im))
        return LCT_ERR_ARG;
    if (hypot(z_re, z_im) > 1.0 + 1e-12)
        return LCT_ERR_DOMAIN;
    if (batch == 0)
        return LCT_OK;
    const bool fp64 = p->prec == LCT_FP64;
    const uintptr_t al = fp64 ? 16 : 8;
    if (in == nullptr || out == nullptr || ((uintptr_t)in) % al || ((uintptr_t)out) % al)
        return LCT_ERR_ARG;
    if (ws == nullptr || ((uintptr_t)ws) % 16 || ws_bytes < ws_bytes_of(p->N, fp64, batch))
        return LCT_ERR_WORKSPACE;
    if ((batch + XS - 1) / XS * ((p->N + XC - 1) / XC) > INT32_MAX)
        return LCT_ERR_ARG;
    const hipError_t e = fp64 ? xft_launch<double>(p, z_re, z_im, in, out, batch, ws, stream)
                         : p->prec == LCT_FP32_SPLITBF16 ? xft_launch_sb(p, z_re, z_im, in, out, batch, ws, stream)
                                                         : xft_launch<float>(p, z_re, z_im, in, out, batch, ws, stream);
    return e == hipSuccess ? LCT_OK : LCT_ERR_HIP;
}

} // extern "C"
