// lct_check.hip - device-side validity check of per-signal parameters that
// live in device memory (matrices M4, fractional orders Z2, ragged
// descriptors): one work-group counts the invalid rows and finds the first,
// with the same rules the host applies to parameters it can see
// (lct_params.hpp).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lct.h"
#include "lct_params.hpp"

using namespace lctk;

namespace {

constexpr int CHECK_THREADS = 1024;
enum { ROWS_M4 = 0, ROWS_Z2 = 1, ROWS_DESC = 2 };

__device__ bool length_ok(int64_t n)
{
    if (n < 1 || n > (int64_t(1) << 24))
        return false;
    while (n % 2 == 0)
        n /= 2;
    while (n % 3 == 0)
        n /= 3;
    while (n % 5 == 0)
        n /= 5;
    return n == 1;
}

__device__ bool m4_ok(const double *r) { return lct_row_finite(r[0], r[1], r[2], r[3]) && lct_row_unimodular(r[0], r[1], r[2], r[3]); }
__device__ bool z2_ok(const double *r) { return frft_row_finite(r[0], r[1]) && frft_row_in_disc(r[0], r[1]); }

__device__ bool desc_ok(const lct_desc &d)
{
    if (d.offset < 0 || d.prec != LCT_FP32 || d.pad != 0 || !length_ok(d.N))
        return false;
    if (d.kind == LCT_KIND_LCT)
        return m4_ok(d.p);
    if (d.kind == LCT_KIND_FRFT)
        return z2_ok(d.p);
    return false;
}

// One work-group of CHECK_THREADS threads; status = {count, first invalid or -1}.
template <int ROWS>
__global__ __launch_bounds__(CHECK_THREADS) void k_check(const double *P, const lct_desc *D, int64_t n, int64_t *status)
{
    __shared__ int64_t cnt[CHECK_THREADS];
    __shared__ int64_t first[CHECK_THREADS];
    const int t = (int)threadIdx.x;
    int64_t c = 0, f = n; // each thread visits increasing rows: its first hit is its smallest
    for (int64_t i = t; i < n; i += CHECK_THREADS) {
        bool ok;
        if constexpr (ROWS == ROWS_M4)
            ok = m4_ok(P + 4 * i);
        else if constexpr (ROWS == ROWS_Z2)
            ok = z2_ok(P + 2 * i);
        else
            ok = desc_ok(D[i]);
        if (!ok) {
            if (c == 0)
                f = i;
            ++c;
        }
    }
    cnt[t] = c;
    first[t] = f;
    __syncthreads();
    for (int w = CHECK_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) {
            cnt[t] += cnt[t + w];
            first[t] = first[t + w] < first[t] ? first[t + w] : first[t];
        }
        __syncthreads();
    }
    if (t == 0) {
        status[0] = cnt[0];
        status[1] = cnt[0] > 0 ? first[0] : -1;
    }
}

int launch_check(int rows, const double *P, const lct_desc *D, int64_t n, int64_t *status, hipStream_t s)
{
    if (rows == ROWS_M4)
        hipLaunchKernelGGL(k_check<ROWS_M4>, dim3(1), dim3(CHECK_THREADS), 0, s, P, D, n, status);
    else if (rows == ROWS_Z2)
        hipLaunchKernelGGL(k_check<ROWS_Z2>, dim3(1), dim3(CHECK_THREADS), 0, s, P, D, n, status);
    else
        hipLaunchKernelGGL(k_check<ROWS_DESC>, dim3(1), dim3(CHECK_THREADS), 0, s, P, D, n, status);
    return hipGetLastError() == hipSuccess ? LCT_OK : LCT_ERR_HIP;
}

} // namespace

extern "C" {

int lct_check_params(int kind, const double *P, int64_t batch, int64_t *status, hipStream_t stream)
{
    if (kind != LCT_KIND_LCT && kind != LCT_KIND_FRFT)
        return LCT_ERR_ARG;
    if (batch < 0 || status == nullptr || ((uintptr_t)status) % 8 || (batch > 0 && P == nullptr) ||
        ((uintptr_t)P) % 8)
        return LCT_ERR_ARG;
    return launch_check(kind == LCT_KIND_LCT ? ROWS_M4 : ROWS_Z2, P, nullptr, batch, status, stream);
}

int lct_check_desc(const lct_desc *d_desc, int64_t nsig, int64_t *status, hipStream_t stream)
{
    if (nsig < 0 || status == nullptr || ((uintptr_t)status) % 8 || (nsig > 0 && d_desc == nullptr) ||
        ((uintptr_t)d_desc) % 8)
        return LCT_ERR_ARG;
    return launch_check(ROWS_DESC, nullptr, d_desc, nsig, status, stream);
}

} // extern "C"
