/*
 * lct.h - C ABI of the MI355X (gfx950) fast discrete linear canonical
 * transform of R. G. Campos and J. Figueroa, "A fast algorithm for the linear
 * canonical transform" (arXiv:0912.1379).
 *
 * Notation (0-based indices j, k in [0, N)):
 *   n_k  = 2k - N + 1
 *   h    = pi / sqrt(2N)                                  eq. (deltk)
 *   x_k  = h n_k / 2          input nodes                 eq. (asymcer)
 *   y_j  = 4 b x_j / pi       output nodes (b != 0)       Algorithm, §3
 *   y_j  = x_j / d            output nodes (b == 0)       §1 definition
 *
 * Data layout: complex samples interleaved {re, im}; FP32 paths use 8-byte
 * complex64, the FP64 path 16-byte complex128.  A batch is `batch` signals of N
 * samples stored contiguously (signal s occupies elements [s*N, (s+1)*N)).
 * Every `in`, `out`, parameter and workspace pointer is DEVICE memory owned by
 * the caller, unless the comment says host.  `in == out` is allowed for the
 * single-pass LCT sizes (a signal's input is read before any of its output is
 * written); the two-pass sizes and the fractional transform need in != out.
 *
 * Execution is asynchronous on `stream` (a hipStream_t; NULL means the
 * default stream).  The library never synchronises and never allocates device
 * memory inside an exec call.  Argument errors are detected on the host before
 * anything is enqueued and reported by the return code; nothing is written.
 * No C++ exception crosses this interface.
 *
 * Supported sizes: N = 2^p 3^q 5^r with 1 <= N <= 2^24.  Sizes up to the LDS
 * limit (FP32: 16384 points, FP64: 8192) run as one pass per signal; larger
 * sizes use a two-pass (four-step) FFT through `out` (then in != out is
 * required).
 */
#ifndef LCT_MI355X_H
#define LCT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
enum {
    LCT_OK = 0,
    LCT_ERR_ARG = -1,            /* null pointer, batch < 0, bad enum, misalignment */
    LCT_ERR_NOT_UNIMODULAR = -2, /* |ad - bc - 1| > 1e-10 max(1, |ad|, |bc|) */
    LCT_ERR_UNSUPPORTED_N = -3,  /* N not 2^p 3^q 5^r or outside [1, 2^24] */
    LCT_ERR_DOMAIN = -4,         /* fractional order |z| > 1 */
    LCT_ERR_WORKSPACE = -5,      /* workspace missing or too small */
    LCT_ERR_HIP = -6,            /* a HIP runtime call failed */
    LCT_ERR_UNSUPPORTED = -7     /* valid request this build does not run */
};

/* Precision selector.  Entry points take any int-sized value here and reject
 * the ones not listed with LCT_ERR_ARG; C++ callers see a fixed underlying
 * type so that such values are representable. */
typedef enum
#ifdef __cplusplus
    : int
#endif
{
    LCT_FP32 = 0,          /* complex64 data, FP32 FFT, FP64 phase reduction */
    LCT_FP64 = 1,          /* complex128 data, FP64 throughout */
    LCT_FP32_SPLITBF16 = 2 /* complex64 data; the FFT's radix-16 stages run on the
                              matrix cores as complex 16 x 16 DFT products with
                              operands split into two BF16 parts (x = hi + lo,
                              W x ~ W_hi x_hi + W_hi x_lo + W_lo x_hi) and FP32
                              accumulation, about 16 significant bits per
                              product; other stages, twiddles and chirps as
                              LCT_FP32.  LCT only (forward and adjoint), N a
                              power of two from 256 to 2^24; other requests
                              return LCT_ERR_UNSUPPORTED. */
} lct_precision;

typedef struct lct_plan_s *lct_plan;

/*
 * Creates an immutable plan for one size and one matrix M = (a b; c d) with
 * ad - bc = 1 (§1).  All per-plan constants are derived here in FP64 /
 * extended precision: the pre-chirp a x_k^2/(2b) and post-chirp d y_j^2/(2b)
 * coefficients (Algorithm, steps 1 and 2), the index phases of eq. (dislctn)
 * and the amplitude h (2 pi i b)^(-1/2) on the principal branch.
 * The plan holds no device memory.  *out is set to NULL on error.
 * c is used only when b == 0 (it is redundant otherwise).
 */
int lct_plan_create(lct_plan *out, int64_t N, double a, double b, double c, double d);
int lct_plan_create_ex(lct_plan *out, int64_t N, double a, double b, double c, double d,
                       lct_precision prec);
/*
 * Plan for samples taken on the scaled input grid xi_k = s x_k, s > 0 finite
 * (the first "scaling" of the scaling-chirp-DFT-chirp-scaling form, §1 and
 * §3): out[j] approximates G(y_j) at y_j = 4 b x_j / (pi s) for b != 0, and
 * y_j = s x_j / d for b == 0 (lct_nodes_scaled).  It is the Riemann sum of
 * the integral of §1 with weight s h:
 *   out[j] = s h (2 pi i b)^(-1/2) sum_k exp(i [a xi_k^2 - 2 xi_k y_j + d y_j^2]/(2b)) in[k],
 * the same DFT with the pre-chirp a s^2 x_k^2/(2b), the post-chirp
 * d y_j^2/(2b) at the scaled y_j, and the amplitude times s, all derived
 * here in extended precision (one set of constants per plan).  This lets one
 * transform read another's output without resampling: after a transform with
 * parameter b1 > 0 the samples lie on s = 4 b1 / pi (for b1 < 0, reverse them
 * first: they lie on s = 4 |b1| / pi in descending order).  s == 1 is
 * lct_plan_create_ex.  lct_exec and lct_exec_adjoint take the scale into
 * account; frft_exec / frft_exec_ws return LCT_ERR_UNSUPPORTED for s != 1.
 * Errors: those of lct_plan_create_ex; LCT_ERR_ARG if s is not a finite
 * positive number or the scaled constants overflow.  *out is NULL on error.
 */
int lct_plan_create_scaled(lct_plan *out, int64_t N, double a, double b, double c, double d, double s,
                           lct_precision prec);
void lct_plan_destroy(lct_plan p);

/*
 * Discrete LCT of `batch` signals (Algorithm, eq. algfxft1):
 *   b != 0:  out[j] = amp * e^{i pi (N-1) j / N} e^{i d y_j^2/(2b)}
 *                      * sum_k e^{-2 pi i j k / N} e^{i pi (N-1) k / N} e^{i a x_k^2/(2b)} in[k],
 *            amp = h (2 pi i b)^(-1/2) e^{-i pi (N-1)^2/(2N)},
 *            which equals the Riemann sum of the integral of §1 at y_j;
 *            out[j] approximates G(4 b x_j / pi).
 *   b == 0:  out[j] = sqrt(d) e^{i c x_j^2/(2d)} in[j]   (§1, f(d y_j) = f(x_j)).
 * The DFT sign is the one of the integral (exp(-i x y / b)); the Algorithm box
 * prints the opposite sign, which returns G at -y_j.
 */
int lct_exec(lct_plan p, const void *in, void *out, int64_t batch, hipStream_t stream);

/*
 * Same transform with one matrix per signal: M4 is DEVICE memory holding
 * batch x 4 doubles (a, b, c, d) in that order.  M4 is not validated on the
 * host (it lives on the device); rows with b == 0 take the diagonal path.
 * This extends the paper's single-matrix statement to a batch.
 */
int lct_exec_many(int64_t N, lct_precision prec, const double *M4, const void *in, void *out,
                  int64_t batch, hipStream_t stream);

/*
 * Adjoint (conjugate transpose) of the b != 0 transform:
 *   out = L^H g,  L^H = (pi / (4|b|)) L^{-1}   (the matrix is unitary up to
 * sqrt(4|b|/pi), §5).  This is the input gradient of a real loss in the
 * complex-gradient convention grad_in = L^H grad_out.
 * Returns LCT_ERR_UNSUPPORTED for plans with b == 0.
 */
int lct_exec_adjoint(lct_plan p, const void *g, void *out, int64_t batch, hipStream_t stream);
int lct_exec_many_adjoint(int64_t N, lct_precision prec, const double *M4, const void *g,
                          void *out, int64_t batch, hipStream_t stream);

/*
 * Parameter gradient of a real loss l, per signal:
 *   grad4[s] = (dl/da, dl/db, dl/dc, dl/dd),  dl/dtheta = Re sum_j conj(g_j) dG_j/dtheta,
 * g = dl/dRe G + i dl/dIm G (DEVICE, batch x N complex), f the forward input.
 * b != 0: the Riemann sum of §1 with the output nodes y_j moving with b;
 * dl/dc = 0 since c does not enter.  b == 0: the diagonal of §1,
 * G_j = sqrt(d) e^{i c x_j^2/(2d)} f_j with output nodes x_j/d moving with d, so
 * dl/da = dl/db = 0 and dl/dc, dl/dd are its derivatives (the discrete matrix
 * has no derivative across b = 0: its nodes 4 b x_j / pi collapse there).
 * The per-signal sums are reduced in a fixed order: results are reproducible
 * bit for bit.  grad4 is DEVICE memory of batch x 4 doubles.  Single-pass
 * lengths only (N <= lct_max_single_pass(prec)); longer ones give
 * LCT_ERR_UNSUPPORTED.  LCT_FP32_SPLITBF16 gives LCT_ERR_UNSUPPORTED.
 */
int lct_param_grad_many(int64_t N, lct_precision prec, const double *M4, const void *f,
                        const void *g, double *grad4, int64_t batch, hipStream_t stream);

/*
 * Same-grid discrete fractional Fourier transform of eqs. (fasy), (primcuad),
 * (cuadtrfor), y_j = x_j, for complex order |z| <= 1:
 *   out[j] = sum_k h sqrt(2/(1-z^2)) exp(-[(1+z^2)(x_j^2+x_k^2) - 4 z x_j x_k]/(2(1-z^2))) in[k].
 * Evaluated as Gaussian-chirp diagonal * FFT convolution * diagonal with every
 * factor of modulus <= 1.  z = 1 and z = -1 return the continuum limits
 * sqrt(2 pi) in[j] and sqrt(2 pi) in[N-1-j].  |z| > 1 + 1e-12 gives
 * LCT_ERR_DOMAIN; orders with 1 < |z| <= 1 + 1e-12 are taken on the unit
 * circle (z / |z|).  Only N and the precision of the plan are used.
 */
int frft_exec(lct_plan p, double z_re, double z_im, const void *in, void *out, int64_t batch,
              hipStream_t stream);
/* One order per signal: Z2 is DEVICE memory of batch x 2 doubles (re, im). */
int frft_exec_many(int64_t N, lct_precision prec, const double *Z2, const void *in, void *out,
                   int64_t batch, hipStream_t stream);

/*
 * Workspace: a caller-owned DEVICE buffer (16-byte aligned) of
 * frft_workspace_size(N, prec, batch) bytes.
 *  - 2N above the single-pass limit: the convolution runs as two-pass FFTs
 *    through 2 x 2N complex samples per signal (the data's and the kernel's
 *    spectra; the first also holds the inverse transform's intermediate).
 *    Required: without enough workspace the calls return LCT_ERR_WORKSPACE
 *    and do nothing.  With one order for the batch (frft_exec_ws) the
 *    kernel's spectrum is computed once, in the first signal's kernel
 *    region, and read by every signal.
 *  - Single pass: 2N complex samples, optional.  frft_exec_ws with such a
 *    workspace computes the DFT of the Gaussian-chirp kernel once for the
 *    whole batch (its order is shared) and every signal reuses it: two
 *    length-2N FFTs per signal instead of three.  Without it (or in
 *    frft_exec / frft_exec_many[_ws], whose orders may differ per signal)
 *    each signal transforms the kernel itself.  The results agree to rounding.
 * in != out is required.
 */
size_t frft_workspace_size(int64_t N, lct_precision prec, int64_t batch);
int frft_exec_ws(lct_plan p, double z_re, double z_im, const void *in, void *out, int64_t batch,
                 void *ws, size_t ws_bytes, hipStream_t stream);
int frft_exec_many_ws(int64_t N, lct_precision prec, const double *Z2, const void *in, void *out,
                      int64_t batch, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * frft_exec_ws without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the workspace is a library-owned static device
 * array of LCT_NOALLOC_SCRATCH_BYTES per device (obtained once per device,
 * held until the process ends).  The call allocates nothing.  Same transform,
 * arguments and errors as frft_exec; a batch whose workspace,
 * frft_workspace_size(N, prec, batch), exceeds LCT_NOALLOC_SCRATCH_BYTES gives
 * LCT_ERR_WORKSPACE (FP32: e.g. 32 signals at N = 65536, 128 at 16384; single-pass
 * lengths need only 2N complex values for any batch).  Every call on one
 * device shares that device's array: calls that overlap in time on one device
 * (different streams, or different host threads) race and must be serialised
 * by the caller.  Nothing in the array needs to start at zero.
 */
#define LCT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int frft_exec_noalloc(lct_plan p, double z_re, double z_im, const void *in, void *out, int64_t batch,
                      hipStream_t stream);

/*
 * LCT of §1 for a complex matrix (a, b, d complex, b != 0; c follows from
 * ad - bc = 1 and does not enter), e.g. damped LCTs, with the output on the
 * input grid (y_j = x_j, eq. asymcer), as the Riemann sum of the integral:
 *   out[j] = h (2 pi i b)^(-1/2) sum_k exp(i [a x_k^2 - 2 x_k x_j + d x_j^2]/(2b)) in[k]
 * (principal root).  For a = d = (z + 1/z)/2, b = i (z - 1/z)/2 this is
 * frft_exec's transform divided by sqrt(2 pi / z).  Computed exactly (up to
 * rounding) as chirp * Gaussian-chirp convolution * chirp in the Toeplitz
 * form, or, input reversed, the Hankel form, whichever has all three factors
 * of modulus <= 1; a matrix for which neither does (the sum would add and
 * cancel exponentially large terms) gives LCT_ERR_DOMAIN.  With conj(b)
 * written b*, the accepted domain is
 *   Toeplitz:  Im b <= 0,  Im[(a - 1) b*] >= 0,  Im[(d - 1) b*] >= 0,   or
 *   Hankel:    Im b >= 0,  Im[(a + 1) b*] >= 0,  Im[(d + 1) b*] >= 0
 * (each up to a relative slack of 1e-12; the factors are i(a -+ 1)/(2b),
 * +-i/(2b) and i(d -+ 1)/(2b), and Re(i q/(2b)) = -Im(q b*)/(2|b|^2)).  Real
 * matrices always qualify (unit-modulus chirps); the bilateral Laplace matrix
 * (0, i, i, 0), whose kernel e^{-x y} has no bounded splitting on a real
 * grid, does not.  One matrix per call: its
 * convolution kernel's spectrum is computed once for the batch when a
 * workspace is given (always, for two-pass lengths).  Workspace, alignment and in != out as frft_exec_ws
 * (frft_workspace_size).  b == 0 and LCT_FP32_SPLITBF16 give
 * LCT_ERR_UNSUPPORTED.
 */
int lct_same_grid_exec(int64_t N, lct_precision prec, double a_re, double a_im, double b_re, double b_im,
                       double d_re, double d_im, const void *in, void *out, int64_t batch, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/*
 * LCT of §1 for a complex matrix (a, b, d complex, b != 0; c follows from
 * ad - bc = 1 and does not enter), evaluated by the Algorithm as printed with
 * complex parameters: input on x_k, output at the complex nodes
 * y_j = 4 b x_j / pi (lct_complex_nodes), as the Riemann sum of the integral
 *   out[j] = h (2 pi i b)^(-1/2) sum_k exp(i [a x_k^2 - 2 x_k y_j + d y_j^2]/(2b)) in[k].
 * The cross term -x_k y_j / b = -4 x_k x_j / pi is real for every b, so the
 * DFT and its index phases are those of the real case; the pre- and
 * post-diagonals become Gaussian chirps exp(i (a/b) x_k^2 / 2) and
 * exp(i b d n_j^2 / N).  Accepted when both have modulus <= 1:
 * Im(a/b) >= 0 and Im(b d) >= 0 (relative slack 1e-12), else
 * LCT_ERR_DOMAIN.  The bilateral Laplace transform, the abstract's special
 * case with kernel e^{-x y}, is (a, b, d) = (0, i, 0): out[j] =
 * (-2 pi)^(-1/2) h sum_k e^{-x_k y_j} in[k] on the imaginary axis
 * y_j = 4 i x_j / pi.  One matrix per call; single-pass lengths
 * (lct_max_single_pass) else LCT_ERR_UNSUPPORTED; b = 0 and
 * LCT_FP32_SPLITBF16 give LCT_ERR_UNSUPPORTED.  in == out allowed.
 * lct_complex_nodes: host helper, y (HOST, 2N doubles, interleaved complex).
 */
int lct_complex_exec(int64_t N, lct_precision prec, double a_re, double a_im, double b_re, double b_im, double d_re,
                     double d_im, const void *in, void *out, int64_t batch, hipStream_t stream);
int lct_complex_nodes(int64_t N, double b_re, double b_im, double *y);

/*
 * Aliasing-aware discrete LCT (b != 0).  The Algorithm samples f on x_k (step
 * h = pi / sqrt(2N)); the pre-chirp e^{i a x^2/(2b)} has local frequency
 * |a/b| |x|, so where |a/b| |x| plus f's own bandwidth passes the grid's
 * Nyquist limit pi / h = sqrt(2N) the sum aliases and no longer approximates
 * the integral of §1 (at the edge |x| = x_max this happens for |a/b| > 4/pi).
 * This mode first interpolates the samples trigonometrically onto the grid of
 * step h / P over the same span,
 *   f(x) = sum_n c_n e^{2 pi i n (x - x_0) / (N h)},  c_n = (1/N) sum_k f_k e^{-2 pi i n k / N},
 * n from -N/2 to N/2 (for even N the coefficient of n = -N/2 split in halves
 * between -N/2 and +N/2), then takes the Riemann sum of §1 on that grid (the
 * scaled grid of lct_plan_create_scaled with P N points and s = 1 / sqrt(P),
 * whose Nyquist limit is P times higher) and returns it at the Algorithm's
 * output nodes y_j = 4 b x_j / pi, the middle N of its P N outputs:
 *   out[j] = (h/P) (2 pi i b)^(-1/2) sum_m exp(i [a xi_m^2 - 2 xi_m y_j + d y_j^2]/(2b)) f(xi_m),
 *   xi_m = (h/P)(m - (P N - 1)/2).
 * P = 1 or b = 0 is lct_exec.  Requirements: a plan of LCT_FP32 or LCT_FP64
 * on the Algorithm's grid (not scaled; else LCT_ERR_UNSUPPORTED), P >= 1 with
 * (P - 1) N even (else LCT_ERR_ARG), P N of the form 2^a 3^b 5^c
 * (LCT_ERR_UNSUPPORTED_N), within the single-pass limit (lct_max_single_pass)
 * and with every prime factor of P dividing N (the two DFTs of the
 * interpolation share one thread layout); else LCT_ERR_UNSUPPORTED.  ws: DEVICE, 16-byte
 * aligned, lct_oversampled_workspace_size(N, P, prec, batch) bytes (the P N
 * fine samples per signal; LCT_ERR_WORKSPACE if smaller; required even where
 * the common (N, P N) pairs run in one kernel whose fine samples stay on chip
 * and leave it untouched).  in == out allowed.
 */
size_t lct_oversampled_workspace_size(int64_t N, int P, lct_precision prec, int64_t batch);
int lct_exec_oversampled(lct_plan p, int P, const void *in, void *out, int64_t batch, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/*
 * Ragged batch in one persistent launch: signals of different lengths, each
 * an LCT with its own matrix or a same-grid fractional transform with its own
 * order.  This extends the paper's single-transform statement to a batch.
 *
 * A descriptor per signal (the same array on the host for planning and on
 * the device for execution; sizes, kinds and offsets must agree, the
 * parameters p may change between executions):
 *   offset  element offset of the signal in `in` and `out` (complex64)
 *   N       its length, of the form 2^k, 3 2^k or 5 2^k; short signals run
 *           in LDS, long ones as a four-step FFT inside one work-group whose
 *           two factors (of N, or of 2N for the fractional transform) must
 *           have that form too (up to N = 2^24 for the LCT); other lengths
 *           give LCT_ERR_UNSUPPORTED
 *   kind    LCT_KIND_LCT: p = (a, b, c, d), ad - bc = 1;
 *           LCT_KIND_FRFT: p = (re z, im z, -, -), |z| <= 1
 * The plan validates the host descriptors, groups short signals of one length
 * into work items, sorts the items by estimated cost (largest first) and
 * keeps the item list in plan-owned device memory.  lct_exec_ragged launches
 * one persistent kernel whose work-groups take items from a counter in the
 * workspace until none is left; the launch (counter reset + kernel) is
 * recorded once per (d_desc, in, out, ws) into a HIP graph and replayed.
 * FP32 only; in != out; the workspace (256-byte aligned, DEVICE) holds the
 * counter and the spectra of long fractional transforms.
 */
enum { LCT_KIND_LCT = 0, LCT_KIND_FRFT = 1 };
typedef struct {
    int64_t offset; /* element offset in `in` and `out` */
    int32_t N;      /* length */
    int32_t kind;   /* LCT_KIND_LCT or LCT_KIND_FRFT */
    int32_t prec;   /* lct_precision; must equal the plan's (LCT_FP32) */
    int32_t pad;    /* reserved, must be 0 */
    double p[4];    /* (a, b, c, d) or (re z, im z, 0, 0) */
} lct_desc;
typedef struct lct_ragged_s *lct_ragged_plan;
int lct_ragged_plan_create(lct_ragged_plan *out, const lct_desc *h_desc, int64_t nsig, lct_precision prec);
size_t lct_ragged_workspace_size(lct_ragged_plan p);
/*
 * Workspace bytes lct_exec_ragged needs for these HOST descriptors (the same
 * value lct_ragged_workspace_size returns for a plan made from them), without
 * making a plan: 256 bytes of counter, then 2 x 2N complex64 samples per
 * fractional transform too long for one work-group's LDS.  The descriptors are
 * validated as by lct_ragged_plan_create (the precision is that of the first
 * descriptor; all must agree); on error *bytes is 0 and the code is returned.
 */
int lct_workspace_size(const lct_desc *h_desc, int64_t nsig, size_t *bytes);
/* Host query: number of work items, persistent grid size, dynamic LDS bytes. */
int lct_ragged_info(lct_ragged_plan p, int *nitems, int *grid, size_t *lds_bytes);
int lct_exec_ragged(lct_ragged_plan p, const lct_desc *d_desc, const void *in, void *out, void *ws,
                    size_t ws_bytes, hipStream_t stream);
void lct_ragged_plan_destroy(lct_ragged_plan p);

/*
 * Device-side check of per-signal parameters that live on the device and so
 * are not validated on the host (lct_exec_many, the adjoints and the
 * parameter gradient: M4; frft_exec_many[_ws]: Z2; lct_exec_ragged: the
 * descriptors).  A row is invalid when
 *   LCT_KIND_LCT (M4 rows a, b, c, d): an entry is not finite, or
 *     |ad - bc - 1| > 1e-10 max(1, |ad|, |bc|) (§1; this includes b = d = 0,
 *     for which the transform divides by zero);
 *   LCT_KIND_FRFT (Z2 rows re z, im z): a part is not finite, or
 *     |z| > 1 + 1e-12 (the quadrature of eq. eqifft needs |z| <= 1);
 *   descriptors: the same per kind, plus an unknown kind, N outside
 *     [1, 2^24] or not 2^p 3^q 5^r, a negative offset, a precision other
 *     than LCT_FP32 or pad != 0.
 * The transforms do not check these rows: an invalid row gives NaN or
 * meaningless output for that signal only.
 * status: DEVICE memory of two int64: status[0] = the number of invalid rows,
 * status[1] = the index of the first invalid row (or -1).  Both are written
 * by one small kernel on `stream` (no memset, no host synchronisation), so
 * the check can sit in the same stream or graph as the transform.  P and
 * d_desc 8-byte aligned; batch/nsig >= 0 (0 writes {0, -1}).
 */
int lct_check_params(int kind, const double *P, int64_t batch, int64_t *status, hipStream_t stream);
int lct_check_desc(const lct_desc *d_desc, int64_t nsig, int64_t *status, hipStream_t stream);

/*
 * Autotuner.  The launch geometry of a transform (values per thread, signals
 * per work-group and the radix order of the FFT stages; for two-pass sizes the
 * split N = N1 N2 and the column and row tile widths) comes from a
 * process-wide table keyed by (kind, N, precision) when it holds an entry,
 * otherwise from a built-in heuristic.  It applies to lct_exec,
 * lct_exec_many, the adjoints and the fractional transform (whose geometry is
 * that of its length-2N convolution); results do not depend on it beyond
 * rounding.
 *
 * lct_autotune times every candidate geometry on the current device (ten
 * launches each after two warm-ups, on `batch` signals of scratch device
 * memory that it allocates and frees; batch 0 means about 2^24 samples),
 * records the fastest in the table and fills *res (may be NULL).  It
 * synchronises `stream`.  A single-pass fractional-transform geometry serves
 * both of its modes (an order per signal, and one order whose kernel spectrum
 * is computed once), so there a candidate's time, and best_us / default_us,
 * is the sum of one execution in each mode.  Entries are single text lines,
 *   lct N=4096 prec=fp32 E=16 S=1 rad=16.16.16
 *   lct N=1048576 prec=fp32 N1=1024 E1=16 E2=16 C=16 RR=16 rad1=16.16.4 rad2=16.16.4
 * ("frft" for the fractional transform); every field is validated against
 * the kernels' preconditions, and an invalid line gives LCT_ERR_ARG.
 *   lct_tune_candidates  the candidate lines, '\n'-separated, into buf (host)
 *   lct_tune_get         the line in use for (kind, N, precision) (host)
 *   lct_tune_set         records one line (host)
 *   lct_tune_load/save   reads / writes a file of lines ('#' comments); a file
 *                        with any invalid line (or a line over 511 bytes) is
 *                        rejected as a whole; a field given twice is invalid
 *   lct_tune_clear       empties the table
 *
 * Environment (read at each use):
 *   LCT_TUNE_CACHE=path  the table is loaded from `path` before the first
 *                        lookup (and again if the variable changes); a
 *                        missing or invalid file leaves the table unchanged.
 *                        Every successful lct_autotune writes the whole table
 *                        back (to a temporary file renamed over `path`).
 *   LCT_AUTOTUNE=1       plan creation (FP32 and FP64 plans) runs
 *                        lct_autotune for both transforms of the plan's
 *                        length on the default stream with batch 0 unless the
 *                        table already holds them; plan creation then
 *                        allocates, synchronises and takes up to seconds.  A
 *                        failed autotune leaves the heuristic.
 */
enum { LCT_TUNE_LCT = 0, LCT_TUNE_FRFT = 1 };
typedef struct {
    int32_t kind;       /* LCT_TUNE_LCT or LCT_TUNE_FRFT */
    int32_t candidates; /* geometries timed */
    double best_us;     /* mean time of one execution with the chosen geometry */
    double default_us;  /* same with the heuristic's geometry */
    int64_t batch;      /* signals per timed execution */
    char config[160];   /* the chosen entry line */
} lct_tune_result;
int lct_autotune(int64_t N, lct_precision prec, int kind, int64_t batch, hipStream_t stream, lct_tune_result *res);
int lct_tune_candidates(int64_t N, lct_precision prec, int kind, char *buf, size_t cap, int *count);
int lct_tune_get(int64_t N, lct_precision prec, int kind, char *buf, size_t cap);
int lct_tune_set(const char *line);
int lct_tune_load(const char *path);
int lct_tune_save(const char *path);
void lct_tune_clear(void);

/*
 * Exact-node discrete fractional transform of §2, eq. (tmat), for a batch of
 * signals sampled at the N zeros x_0 < ... < x_{N-1} of H_N (not the
 * asymptotic nodes of eq. asymcer):
 *   out[s] = F_z in[s],  F_z = sqrt(2 pi) U^T D(z) U,  D(z) = diag(1, z, ..., z^(N-1)),
 * U the orthogonal matrix of eq. (ortvec), U[n][k] = (u_k)_n.  This is the
 * O(N^2)-per-signal method the fast transforms approximate; it is evaluated as
 * two dense products on the matrix cores, FP64 or FP32 arithmetic by the
 * plan's precision; with LCT_FP32_SPLITBF16 the data are complex64 and the
 * products run as BF16 hi + lo parts with FP32 accumulation (about 16
 * significant bits per product).  The weights sqrt(2 pi) z^n are formed on
 * the device in double-double.
 *
 * xft_plan_create computes the zeros (QR eigenvalues of the symmetric
 * tridiagonal H of §2, polished by Newton steps) and U (recurrence of eq.
 * receqg, normalised by the Christoffel-Darboux sum) on the host and keeps U
 * and U^T in plan-owned DEVICE memory (2 N^2 values of the plan's precision,
 * or their BF16 parts with rows padded to a multiple of 8);
 * 1 <= N <= 16384, any N (host time about 1 s at N = 4096, 5 s at 8192, 25 s
 * at 16384, mostly first touches of the N^2 arrays).  xft_exec: in, out DEVICE batch x N complex (in ==
 * out allowed), |z| <= 1 (beyond 1e-12: LCT_ERR_DOMAIN), ws a caller-owned
 * DEVICE workspace of xft_workspace_size(N, prec, batch) bytes, 16-byte
 * aligned (else LCT_ERR_WORKSPACE).  Calls on one plan may run concurrently
 * only with separate workspaces.
 * xft_nodes / xft_vectors are host helpers returning the zeros (N doubles) and
 * U (N x N doubles, row-major) in host memory.
 */
typedef struct xft_plan_s *xft_plan;
int xft_plan_create(xft_plan *out, int64_t N, lct_precision prec);
void xft_plan_destroy(xft_plan p);
size_t xft_workspace_size(int64_t N, lct_precision prec, int64_t batch);
int xft_exec(xft_plan p, double z_re, double z_im, const void *in, void *out, int64_t batch, void *ws,
             size_t ws_bytes, hipStream_t stream);
int xft_nodes(int64_t N, double *x);
int xft_vectors(int64_t N, double *U);

/*
 * Host helper: input nodes x (N doubles, eq. asymcer) and output nodes y
 * (N doubles: 4 b x_j / pi, or x_j / d when b == 0).  Either pointer may be NULL.
 * Host memory.  Returns LCT_ERR_ARG for N < 1 or b == d == 0.
 */
int lct_nodes(int64_t N, double b, double d, double *x, double *y);

/*
 * Host helper for plans on the scaled grid (lct_plan_create_scaled): input
 * nodes x (N doubles, s x_k) and output nodes y (N doubles: 4 b x_k / (pi s),
 * or s x_k / d when b == 0).  Either pointer may be NULL.  Host memory.
 * Returns LCT_ERR_ARG for N < 1, b == d == 0, or s not finite and positive.
 */
int lct_nodes_scaled(int64_t N, double b, double d, double s, double *x, double *y);

/* Static description of a return code. */
const char *lct_strerror(int code);

/* Largest N that runs as a single pass for the precision (host query). */
int64_t lct_max_single_pass(lct_precision prec);

#ifdef __cplusplus
}
#endif

#endif /* LCT_MI355X_H */
