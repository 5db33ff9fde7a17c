/*
 * Oracle for the fast discrete linear canonical transform of
 * R. G. Campos and J. Figueroa, "A fast algorithm for the linear canonical
 * transform" (arXiv:0912.1379).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, direct CPU
 * evaluation of what the paper defines, in FP64 inputs/outputs with
 * long-double (x87 80-bit) internal arithmetic.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  The GPU
 * library shares no code, header, table or constant with it.
 *
 * Conventions (0-based, the paper's 1-based index k maps to k+1):
 *   N          number of samples
 *   n_k        2k - N + 1                                 (odd/even integer)
 *   h          pi / sqrt(2N)                               eq. (deltk)
 *   x_k        h * n_k / 2                                 eq. (asymcer)
 *   y_j        4 b x_j / pi                                Algorithm, §3
 *   complex arrays are interleaved {re, im} doubles.
 *
 * Readings of the paper that this file fixes (each also listed in the design
 * notes of the repository):
 *   - The discrete LCT is the Riemann sum of the integral of §1 on the nodes
 *     x_k with weight h, evaluated at y_j.  The kernel sign is the one of the
 *     integral (exp(-i x y / b) after expanding), which is what the
 *     Algorithm's output claims to approximate.
 *   - (2 pi i b)^(-1/2) and sqrt(d) take the principal branch.
 *   - For b = 0 the output node is y_j = x_j / d, so f(d y_j) = f(x_j).
 *   - The same-grid fractional transform (eqs. fasy, primcuad, cuadtrfor) is
 *     the Riemann sum with y_j = x_j; at z = 1 and z = -1, where 1 - z^2
 *     vanishes, the continuum limits sqrt(2 pi) f(x) and sqrt(2 pi) f(-x)
 *     are returned.
 *
 * Parity status of every function here is listed beside it.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* glibc defines CMPLXL only for GCC; clang (the sanitized build) has the same builtin. */
#ifndef CMPLXL
#define CMPLXL(x, y) __builtin_complex((long double)(x), (long double)(y))
#endif

#define PI_L 3.141592653589793238462643383279502884L

/* Compensated (Neumaier) summation in long double: the running sum s and the
 * rounding error c of every addition so far; the sum is s + c.  Sums of 2^20
 * terms then carry about one rounding of the result instead of up to 2^20. */
typedef struct {
    long double s, c;
} ksum;

static void ksum_add(ksum *k, long double v)
{
    long double t = k->s + v;
    if (fabsl(k->s) >= fabsl(v))
        k->c += (k->s - t) + v;
    else
        k->c += (v - t) + k->s;
    k->s = t;
}

static long double ksum_value(const ksum *k) { return k->s + k->c; }

static long double node_l(int64_t N, int64_t k)
{
    /* eq. (asymcer), 0-based: x_k = (2k - N + 1) pi / (2 sqrt(2N)) */
    return (long double)(2 * k - N + 1) * PI_L / (2.0L * sqrtl(2.0L * (long double)N));
}

/* Nodes x_k of eq. (asymcer).  Pinned: symmetric, equispaced with the
 * spacing of eq. (deltk), compared with the true Hermite zeros for large N. */
void oracle_nodes(int64_t N, double *x)
{
    for (int64_t k = 0; k < N; ++k)
        x[k] = (double)node_l(N, k);
}

/* (2 pi i b)^(-1/2) on the principal branch. */
static long double complex inv_sqrt_2pi_i_b(long double b)
{
    long double complex w = csqrtl(CMPLXL(0.0L, 2.0L * PI_L * b));
    return 1.0L / w;
}

/*
 * O1: discrete LCT as the Riemann sum of the definition of §1, for samples
 * f_k = f(xi_k) taken on the input grid xi_k = s x_k (s > 0; s = 1 is the
 * Algorithm's grid), quadrature weight s h:
 *   G_j = sum_k s h (2 pi i b)^(-1/2) exp(i [a xi_k^2 - 2 xi_k y_j + d y_j^2]/(2b)) f_k,
 * at the output nodes y_j = 4 b x_j / (pi s) (the Algorithm's y_j for s = 1;
 * for other s the nodes that keep the cross term a DFT).  For b = 0 the
 * definition of §1 reads
 *   G(y) = sqrt(d) exp(i c d y^2 / 2) f(d y)
 * and with y_j = xi_j / d this is sqrt(d) exp(i c xi_j^2 / (2d)) f_j.
 *
 * The three phase terms are written in the variables n_j, n_k, which is an
 * exact substitution of xi and y:
 *   a xi_k^2/(2b)  = a s^2 pi^2 n_k^2 / (16 b N)
 *   xi_k y_j / b   = pi n_j n_k / (2N)        (reduced exactly modulo 4N)
 *   d y_j^2/(2b)   = b d n_j^2 / (N s^2)
 * so no phase of magnitude 1e4..1e7 rad is rounded before its reduction.
 *
 * rows == NULL means every row 0..N-1 (then nrows must be N).
 * Returns 0, or -1 on bad arguments.
 * Pinned: closed form eq. (exa1), Hermite-Gauss closed form, unitarity,
 * numpy FFT for a=d=0, b=1, composition law, mpmath brute force; for s != 1
 * the Gaussian closed form on scaled grids and a chain of two transforms
 * against the closed form of the matrix product.
 */
int oracle_lct_rows_scaled(int64_t N, double a, double b, double c, double d, double s,
                           const double *f, const int64_t *rows, int64_t nrows,
                           double *out)
{
    if (N < 1 || f == NULL || out == NULL || nrows < 0 || !(s > 0.0) || !isfinite(s))
        return -1;
    if (rows == NULL && nrows != N)
        return -1;
    const long double h = PI_L / sqrtl(2.0L * (long double)N);
    const long double S = (long double)s;

    if (b == 0.0) {
        if (d == 0.0)
            return -1;
        long double complex sd = csqrtl(CMPLXL((long double)d, 0.0L));
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t j = rows ? rows[r] : r;
            if (j < 0 || j >= N)
                return -1;
            long double xj = node_l(N, j);
            long double ph = (long double)c * S * S * xj * xj / (2.0L * (long double)d);
            long double complex v = sd * cexpl(CMPLXL(0.0L, ph)) *
                                    CMPLXL((long double)f[2 * j], (long double)f[2 * j + 1]);
            out[2 * r] = (double)creall(v);
            out[2 * r + 1] = (double)cimagl(v);
        }
        return 0;
    }

    const long double A = (long double)a, B = (long double)b, D = (long double)d;
    const long double complex amp = S * h * inv_sqrt_2pi_i_b(B);
    /* per-k pre phase a x_k^2/(2b) (hoisted out of the row loop) */
    long double *t1 = (long double *)malloc(sizeof(long double) * (size_t)N);
    if (!t1)
        return -1;
    for (int64_t k = 0; k < N; ++k) {
        long double nk = (long double)(2 * k - N + 1);
        t1[k] = A * S * S * PI_L * PI_L * nk * nk / (16.0L * B * (long double)N);
    }
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t j = rows ? rows[r] : r;
        if (j < 0 || j >= N) {
            bad = 1;
            continue;
        }
        int64_t nj = 2 * j - N + 1;
        long double t3 = B * D * (long double)nj * (long double)nj / ((long double)N * S * S);
        ksum sr = {0.0L, 0.0L}, si = {0.0L, 0.0L};
        for (int64_t k = 0; k < N; ++k) {
            int64_t nk = 2 * k - N + 1;
            int64_t m = (nj * nk) % (4 * N);
            if (m < 0)
                m += 4 * N;
            long double cross = PI_L * (long double)m / (2.0L * (long double)N);
            long double ph = t1[k] - cross + t3;
            long double s, co;
            s = sinl(ph);
            co = cosl(ph);
            long double fr = (long double)f[2 * k], fi = (long double)f[2 * k + 1];
            ksum_add(&sr, co * fr - s * fi);
            ksum_add(&si, co * fi + s * fr);
        }
        long double complex v = amp * CMPLXL(ksum_value(&sr), ksum_value(&si));
        out[2 * r] = (double)creall(v);
        out[2 * r + 1] = (double)cimagl(v);
    }
    free(t1);
    return bad ? -1 : 0;
}

/* The Algorithm's grid (s = 1). */
int oracle_lct_rows(int64_t N, double a, double b, double c, double d,
                    const double *f, const int64_t *rows, int64_t nrows,
                    double *out)
{
    return oracle_lct_rows_scaled(N, a, b, c, d, 1.0, f, rows, nrows, out);
}

/*
 * O4: the LCT of §1 for a complex matrix (a, b, d complex, b != 0; c is
 * implied by ad - bc = 1 and does not enter) as the Riemann sum of its
 * integral on one grid for input and output, y_j = x_j (eq. asymcer):
 *   G_j = sum_k h (2 pi i b)^(-1/2) exp(i [a x_k^2 - 2 x_k x_j + d x_j^2]/(2b)) f_k,
 * the principal branch of the root.  For a = d = (z + 1/z)/2, b = i (z - 1/z)/2
 * this is the same-grid fractional transform of eqs. (fasy)-(cuadtrfor) up to
 * the factor sqrt(2 pi / z).  rows == NULL means every row (nrows must be N).
 * Returns 0, or -1 on bad arguments.
 * Pinned: the fractional transform for a = d, the chirp-DFT-chirp sum O1 for
 * real matrices with b = pi/4 (where the two grids coincide), the complex
 * Gaussian closed form, mpmath brute force.
 */
int oracle_lct_same_rows(int64_t N, double ar, double ai, double br, double bi, double dr, double di,
                         const double *f, const int64_t *rows, int64_t nrows, double *out)
{
    if (N < 1 || f == NULL || out == NULL || nrows < 0 || (br == 0.0 && bi == 0.0))
        return -1;
    if (rows == NULL && nrows != N)
        return -1;
    const long double h = PI_L / sqrtl(2.0L * (long double)N);
    const long double complex A = CMPLXL(ar, ai), B = CMPLXL(br, bi), D = CMPLXL(dr, di);
    const long double complex w = CMPLXL(0.0L, 1.0L) / (2.0L * B); /* i / (2b) */
    const long double complex amp = h / csqrtl(CMPLXL(0.0L, 2.0L * PI_L) * B);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t j = rows ? rows[r] : r;
        if (j < 0 || j >= N) {
            bad = 1;
            continue;
        }
        const long double xj = node_l(N, j);
        ksum ar_ = {0.0L, 0.0L}, ai_ = {0.0L, 0.0L};
        for (int64_t k = 0; k < N; ++k) {
            const long double xk = node_l(N, k);
            const long double complex e = w * (A * xk * xk - 2.0L * xk * xj + D * xj * xj);
            const long double complex t = cexpl(e) * CMPLXL((long double)f[2 * k], (long double)f[2 * k + 1]);
            ksum_add(&ar_, creall(t));
            ksum_add(&ai_, cimagl(t));
        }
        const long double complex v = amp * CMPLXL(ksum_value(&ar_), ksum_value(&ai_));
        out[2 * r] = (double)creall(v);
        out[2 * r + 1] = (double)cimagl(v);
    }
    return bad ? -1 : 0;
}

/*
 * O6: the LCT of §1 for a complex matrix (a, b, d complex, b != 0; c implied
 * by ad - bc = 1) as the Riemann sum of its integral on the Algorithm's input
 * nodes x_k (eq. asymcer) at its output nodes y_j = 4 b x_j / pi, here complex:
 *   G_j = sum_k h (2 pi i b)^(-1/2) exp(i [a x_k^2 - 2 x_k y_j + d y_j^2]/(2b)) f_k,
 * principal branch of the root.  The bilateral Laplace transform is the case
 * (a, b, d) = (0, i, 0): G_j = (-2 pi)^(-1/2) h sum_k e^{-x_k y_j} f_k at
 * y_j = 4 i x_j / pi.  rows == NULL means every row (nrows must be N).
 * Returns 0, or -1 on bad arguments.
 * Pinned: O1 for real matrices, the complex Gaussian integral, the bilateral
 * Laplace transform of a Gaussian in closed form, mpmath brute force.
 */
int oracle_lct_complex_rows(int64_t N, double ar, double ai, double br, double bi, double dr, double di,
                            const double *f, const int64_t *rows, int64_t nrows, double *out)
{
    if (N < 1 || f == NULL || out == NULL || nrows < 0 || (br == 0.0 && bi == 0.0))
        return -1;
    if (rows == NULL && nrows != N)
        return -1;
    const long double h = PI_L / sqrtl(2.0L * (long double)N);
    const long double complex A = CMPLXL(ar, ai), B = CMPLXL(br, bi), D = CMPLXL(dr, di);
    const long double complex w = CMPLXL(0.0L, 1.0L) / (2.0L * B); /* i / (2b) */
    const long double complex amp = h / csqrtl(CMPLXL(0.0L, 2.0L * PI_L) * B);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t j = rows ? rows[r] : r;
        if (j < 0 || j >= N) {
            bad = 1;
            continue;
        }
        const long double complex yj = 4.0L * B * node_l(N, j) / PI_L;
        ksum ar_ = {0.0L, 0.0L}, ai_ = {0.0L, 0.0L};
        for (int64_t k = 0; k < N; ++k) {
            const long double xk = node_l(N, k);
            const long double complex e = w * (A * xk * xk - 2.0L * xk * yj + D * yj * yj);
            const long double complex t = cexpl(e) * CMPLXL((long double)f[2 * k], (long double)f[2 * k + 1]);
            ksum_add(&ar_, creall(t));
            ksum_add(&ai_, cimagl(t));
        }
        const long double complex v = amp * CMPLXL(ksum_value(&ar_), ksum_value(&ai_));
        out[2 * r] = (double)creall(v);
        out[2 * r + 1] = (double)cimagl(v);
    }
    return bad ? -1 : 0;
}

/*
 * Adjoint of the discrete LCT matrix of oracle_lct_rows (b != 0):
 *   (L^H g)_k = sum_j conj(L_jk) g_j.
 * This is the gradient of a real loss with respect to the input samples in
 * the complex-gradient convention grad_f = L^H grad_G.
 * Pinned: <L f, g> = <f, L^H g> with the forward oracle, and unitarity.
 */
int oracle_lct_adjoint(int64_t N, double a, double b, double c, double d,
                       const double *g, double *out)
{
    (void)c;
    if (N < 1 || g == NULL || out == NULL || b == 0.0)
        return -1;
    const long double h = PI_L / sqrtl(2.0L * (long double)N);
    const long double A = (long double)a, B = (long double)b, D = (long double)d;
    const long double complex amp = h * inv_sqrt_2pi_i_b(B);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < N; ++k) {
        int64_t nk = 2 * k - N + 1;
        long double t1 = A * PI_L * PI_L * (long double)nk * (long double)nk /
                         (16.0L * B * (long double)N);
        ksum sr = {0.0L, 0.0L}, si = {0.0L, 0.0L};
        for (int64_t j = 0; j < N; ++j) {
            int64_t nj = 2 * j - N + 1;
            int64_t m = (nj * nk) % (4 * N);
            if (m < 0)
                m += 4 * N;
            long double cross = PI_L * (long double)m / (2.0L * (long double)N);
            long double t3 = B * D * (long double)nj * (long double)nj / (long double)N;
            long double ph = -(t1 - cross + t3); /* conjugate phase */
            long double s = sinl(ph), co = cosl(ph);
            long double gr = (long double)g[2 * j], gi = (long double)g[2 * j + 1];
            ksum_add(&sr, co * gr - s * gi);
            ksum_add(&si, co * gi + s * gr);
        }
        long double complex v = conjl(amp) * CMPLXL(ksum_value(&sr), ksum_value(&si));
        out[2 * k] = (double)creall(v);
        out[2 * k + 1] = (double)cimagl(v);
    }
    return 0;
}

/*
 * Gradient of a real loss l(G) with respect to the real parameters
 * (a, b, c, d) of the b != 0 transform, given g = dl/dRe G + i dl/dIm G:
 *   dl/dtheta = Re sum_j conj(g_j) dG_j/dtheta.
 * dG_j/dtheta differentiates every entry of the dense matrix of
 * oracle_lct_rows, with the output nodes y_j = 4 b x_j / pi moving with b:
 *   phase  Phi_jk = a x_k^2/(2b) - 4 x_j x_k / pi + 8 b d x_j^2 / pi^2
 *   dPhi/da = x_k^2/(2b),  dPhi/db = -a x_k^2/(2 b^2) + 8 d x_j^2/pi^2,
 *   dPhi/dd = 8 b x_j^2 / pi^2,  amplitude h (2 pi i b)^(-1/2): d/db = -1/(2b).
 * c does not enter for b != 0, so dl/dc = 0.
 *
 * For b = 0 the transform is the diagonal of §1, G_j = sqrt(d) exp(i c x_j^2/(2d)) f_j
 * (output nodes x_j / d moving with d, as y_j moves with b above):
 *   dG_j/dc = i x_j^2/(2d) G_j,   dG_j/dd = (1/(2d) - i c x_j^2/(2 d^2)) G_j,
 * and a, b do not enter that formula (a = 1/d there), so dl/da = dl/db = 0.
 * The discrete b != 0 matrix does not tend to the diagonal as b -> 0 (its
 * output nodes 4 b x_j / pi collapse to 0), so no derivative across b = 0 is
 * defined.
 * Pinned: central finite differences of oracle_lct_rows (in a, b, d for
 * b != 0 with c following from ad - bc = 1; in c and d at b = 0).
 */
int oracle_lct_param_grad(int64_t N, double a, double b, double c, double d,
                          const double *f, const double *g, double *grad4)
{
    if (N < 1 || f == NULL || g == NULL || grad4 == NULL)
        return -1;
    if (b == 0.0) {
        if (d == 0.0)
            return -1;
        const long double C = (long double)c, D = (long double)d;
        const long double complex sd = csqrtl(CMPLXL(D, 0.0L));
        long double gc = 0.0L, gd = 0.0L;
        for (int64_t j = 0; j < N; ++j) {
            const long double xj = node_l(N, j);
            const long double x2 = xj * xj;
            const long double complex G = sd * cexpl(CMPLXL(0.0L, C * x2 / (2.0L * D))) *
                                          CMPLXL((long double)f[2 * j], (long double)f[2 * j + 1]);
            const long double complex gj = CMPLXL((long double)g[2 * j], (long double)g[2 * j + 1]);
            gc += creall(conjl(gj) * CMPLXL(0.0L, x2 / (2.0L * D)) * G);
            gd += creall(conjl(gj) * CMPLXL(1.0L / (2.0L * D), -C * x2 / (2.0L * D * D)) * G);
        }
        grad4[0] = 0.0;
        grad4[1] = 0.0;
        grad4[2] = (double)gc;
        grad4[3] = (double)gd;
        return 0;
    }
    const long double h = PI_L / sqrtl(2.0L * (long double)N);
    const long double A = (long double)a, B = (long double)b, D = (long double)d;
    const long double complex amp = h * inv_sqrt_2pi_i_b(B);
    long double ga = 0.0L, gb = 0.0L, gd = 0.0L;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : ga, gb, gd)
    for (int64_t j = 0; j < N; ++j) {
        long double xj = node_l(N, j);
        int64_t nj = 2 * j - N + 1;
        long double complex dA = 0, dB = 0, dD = 0;
        for (int64_t k = 0; k < N; ++k) {
            long double xk = node_l(N, k);
            int64_t nk = 2 * k - N + 1;
            int64_t m = (nj * nk) % (4 * N);
            if (m < 0)
                m += 4 * N;
            long double ph = A * xk * xk / (2.0L * B) -
                             PI_L * (long double)m / (2.0L * (long double)N) +
                             8.0L * B * D * xj * xj / (PI_L * PI_L);
            long double complex e = amp * cexpl(CMPLXL(0.0L, ph)) *
                                    CMPLXL((long double)f[2 * k], (long double)f[2 * k + 1]);
            long double dpa = xk * xk / (2.0L * B);
            long double dpb = -A * xk * xk / (2.0L * B * B) + 8.0L * D * xj * xj / (PI_L * PI_L);
            long double dpd = 8.0L * B * xj * xj / (PI_L * PI_L);
            dA += e * CMPLXL(0.0L, dpa);
            dB += e * (CMPLXL(-1.0L / (2.0L * B), dpb));
            dD += e * CMPLXL(0.0L, dpd);
        }
        long double complex gj = CMPLXL((long double)g[2 * j], (long double)g[2 * j + 1]);
        ga += creall(conjl(gj) * dA);
        gb += creall(conjl(gj) * dB);
        gd += creall(conjl(gj) * dD);
    }
    grad4[0] = (double)ga;
    grad4[1] = (double)gb;
    grad4[2] = 0.0;
    grad4[3] = (double)gd;
    return 0;
}

/*
 * O3: same-grid discrete fractional Fourier transform, the Riemann sum of
 * eqs. (fasy), (primcuad) with y_j = x_j (eq. cuadtrfor):
 *   g_j = sum_k h sqrt(2/(1-z^2))
 *             exp(-[(1+z^2)(x_j^2+x_k^2) - 4 z x_j x_k] / (2(1-z^2))) f_k,
 * |z| <= 1, principal square root.  z = 1 and z = -1 return the continuum
 * limits sqrt(2 pi) f_j and sqrt(2 pi) f_{N-1-j}.  |z| > 1 + 1e-12 returns -2.
 * Pinned: continuum eigen-identity on Hermite functions, z = +-i reduces to
 * the Fourier kernel of eq. (fftuno), mpmath brute force.
 */
int oracle_frft_rows(int64_t N, double zr, double zi, const double *f,
                     const int64_t *rows, int64_t nrows, double *out)
{
    if (N < 1 || f == NULL || out == NULL || nrows < 0)
        return -1;
    if (rows == NULL && nrows != N)
        return -1;
    const long double complex z = CMPLXL((long double)zr, (long double)zi);
    if (cabsl(z) > 1.0L + 1e-12L) /* allow rounding of points on the circle */
        return -2;
    const long double h = PI_L / sqrtl(2.0L * (long double)N);
    const long double s2pi = sqrtl(2.0L * PI_L);
    if (zi == 0.0 && (zr == 1.0 || zr == -1.0)) {
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t j = rows ? rows[r] : r;
            if (j < 0 || j >= N)
                return -1;
            int64_t src = zr > 0 ? j : N - 1 - j;
            out[2 * r] = (double)(s2pi * (long double)f[2 * src]);
            out[2 * r + 1] = (double)(s2pi * (long double)f[2 * src + 1]);
        }
        return 0;
    }
    const long double complex omz2 = 1.0L - z * z;
    const long double complex pref = h * csqrtl(2.0L / omz2);
    const long double complex opz2 = 1.0L + z * z;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t j = rows ? rows[r] : r;
        if (j < 0 || j >= N) {
            bad = 1;
            continue;
        }
        long double xj = node_l(N, j);
        ksum ar_ = {0.0L, 0.0L}, ai_ = {0.0L, 0.0L};
        for (int64_t k = 0; k < N; ++k) {
            long double xk = node_l(N, k);
            long double complex e =
                -(opz2 * (xj * xj + xk * xk) - 4.0L * z * xj * xk) / (2.0L * omz2);
            long double complex t = cexpl(e) * CMPLXL((long double)f[2 * k], (long double)f[2 * k + 1]);
            ksum_add(&ar_, creall(t));
            ksum_add(&ai_, cimagl(t));
        }
        long double complex v = pref * CMPLXL(ksum_value(&ar_), ksum_value(&ai_));
        out[2 * r] = (double)creall(v);
        out[2 * r + 1] = (double)cimagl(v);
    }
    return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* O2: exact Hermite-zero quadrature of §2.                               */
/* ---------------------------------------------------------------------- */

/* Number of eigenvalues of the symmetric tridiagonal H of §2 (zero diagonal,
 * off-diagonal sqrt(n/2), n = 1..N-1) that are smaller than lam: the count of
 * negative pivots of the LDL^T factorisation of H - lam I (Sturm sequence). */
static int64_t sturm_count(int64_t N, long double lam)
{
    int64_t cnt = 0;
    long double q = -lam;
    if (q < 0)
        ++cnt;
    for (int64_t i = 1; i < N; ++i) {
        if (q == 0.0L)
            q = 1e-300L;
        q = -lam - ((long double)i / 2.0L) / q;
        if (q < 0)
            ++cnt;
    }
    return cnt;
}

/* Eigenvalues x_0 < ... < x_{N-1} of H (the zeros of H_N, §2) by bisection
 * on the Sturm count, to full double precision.
 * Pinned: numpy.polynomial.hermite.hermgauss, closed-form zeros N <= 4. */
void oracle_hermite_zeros(int64_t N, double *x)
{
    const long double bound = sqrtl(2.0L * (long double)N) + 1.0L; /* Gershgorin */
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t k = 0; k < N; ++k) {
        long double lo = -bound, hi = bound;
        for (int it = 0; it < 200; ++it) {
            long double mid = 0.5L * (lo + hi);
            if (mid <= lo || mid >= hi)
                break;
            if (sturm_count(N, mid) > k)
                hi = mid;
            else
                lo = mid;
        }
        x[k] = (double)(0.5L * (lo + hi));
    }
}

/*
 * Orthonormal eigenvectors of eq. (ortvec): column k of U (row-major
 * U[n*N + k]) is proportional to (phi_0(x_k), ..., phi_{N-1}(x_k)) with
 * phi_n = H_n / sqrt(2^n n!), i.e. s_{n+1} H_n(x_k).  phi follows from the
 * recurrence eq. (receqg) divided by sqrt(2^(n+1) (n+1)!):
 *   phi_{n+1} = sqrt(2/(n+1)) x phi_n - sqrt(n/(n+1)) phi_{n-1}.
 * Columns are rescaled by powers of two while they grow (they reach
 * e^(x^2/2)), normalised to unit length, and signed so that the last
 * component is (-1)^(N+k) / sqrt(N) in the paper's 1-based k, as eq. (ortvec)
 * gives for n = N.
 * Pinned: U^T U = I, |U[N-1][k]| = 1/sqrt(N), sqrt(pi) U[0][k]^2 equals the
 * Gauss-Hermite weights of numpy hermgauss.
 */
void oracle_hermite_vectors(int64_t N, const double *x, double *U)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t k = 0; k < N; ++k) {
        long double xk = (long double)x[k];
        long double pm1 = 0.0L, p = 1.0L;
        long double *col = (long double *)malloc(sizeof(long double) * (size_t)N);
        col[0] = 1.0L;
        for (int64_t n = 0; n + 1 < N; ++n) {
            long double pn1 = sqrtl(2.0L / (long double)(n + 1)) * xk * p -
                              sqrtl((long double)n / (long double)(n + 1)) * pm1;
            pm1 = p;
            p = pn1;
            col[n + 1] = p;
            if (fabsl(p) > 0x1p1000L) {
                for (int64_t m = 0; m <= n + 1; ++m)
                    col[m] *= 0x1p-1000L;
                p *= 0x1p-1000L;
                pm1 *= 0x1p-1000L;
            }
        }
        long double nrm = 0.0L;
        for (int64_t n = 0; n < N; ++n)
            nrm += col[n] * col[n];
        nrm = sqrtl(nrm);
        /* paper's k is k+1 here: wanted sign of last entry is (-1)^(N+k+1) */
        long double want = ((N + k + 1) % 2 == 0) ? 1.0L : -1.0L;
        long double sg = (col[N - 1] * want >= 0) ? 1.0L : -1.0L;
        for (int64_t n = 0; n < N; ++n)
            U[n * N + k] = (double)(sg * col[n] / nrm);
        free(col);
    }
}

/*
 * Exact discrete fractional transform of eq. (tmat):
 *   F_z = sqrt(2 pi) U^T D(z) U,  D(z) = diag(1, z, ..., z^(N-1)),
 * (F_z)_jk = sqrt(2 pi) sum_n U[n][j] z^n U[n][k]; row-major complex output.
 * Pinned: F_z applied to the rows of U gives sqrt(2 pi) z^n times them;
 * F_z / sqrt(2 pi) is unitary for |z| = 1; F_1 = sqrt(2 pi) I.
 */
void oracle_Fz_exact(int64_t N, const double *U, double zr, double zi, double *F)
{
    const long double complex z = CMPLXL((long double)zr, (long double)zi);
    long double complex *zp = (long double complex *)malloc(sizeof(long double complex) * (size_t)N);
    zp[0] = 1.0L;
    for (int64_t n = 1; n < N; ++n)
        zp[n] = zp[n - 1] * z;
    const long double s2pi = sqrtl(2.0L * PI_L);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t k = 0; k < N; ++k) {
            long double complex acc = 0;
            for (int64_t n = 0; n < N; ++n)
                acc += (long double)U[n * N + j] * zp[n] * (long double)U[n * N + k];
            acc *= s2pi;
            F[2 * (j * N + k)] = (double)creall(acc);
            F[2 * (j * N + k) + 1] = (double)cimagl(acc);
        }
    }
    free(zp);
}

/* Number of OpenMP threads the oracle uses (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads of later calls (for timing on one core).
 * Each output row is summed by one thread, so the rows do not depend on it;
 * only the parameter gradient's reduction over rows is ordered by it. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
