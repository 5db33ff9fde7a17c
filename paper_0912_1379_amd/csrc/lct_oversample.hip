// lct_oversample.hip - launches of the aliasing-aware LCT's own kernels: the
// interpolation onto the finer grid, the window copy, and the fused kernel
// that interpolates, transforms on the fine grid and stores the window in one
// pass (elsewhere the fine-grid transform runs on the LCT kernels).
#include "oversample_impl.hpp"

namespace lctk {

namespace {
template <typename R, int E, int NF1, int NF2>
hipError_t launch_interp_fixed(const void *in, void *ws, const InterpArgs &a, size_t lds, hipStream_t s)
{
    using V = typename Vec<R>::T;
    if (hipError_t r = allow_lds((const void *)k_interp<R, E, NF1, NF2>, lds); r != hipSuccess)
        return r;
    hipLaunchKernelGGL((k_interp<R, E, NF1, NF2>), dim3((unsigned)a.batch), dim3(a.T), lds, s, (const V *)in, (V *)ws,
                       a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_interp_t(int E, const void *in, void *ws, const InterpArgs &a, size_t lds, hipStream_t s)
{
    using V = typename Vec<R>::T;
    // compile-time schedules for the common FP32 (N, P N) pairs
    if constexpr (sizeof(R) == 4) {
        const int M = a.N * a.P;
        if (E == 16 && is_fixed_sched(a.sc1, a.N, 16) && is_fixed_sched(a.sc2, M, 16)) {
#define Y(n, m)                                                                                                      \
    if (a.N == n && M == m)                                                                                          \
        return launch_interp_fixed<R, 16, n, m>(in, ws, a, lds, s);
            Y(1024, 2048) Y(1024, 4096) Y(2048, 4096) Y(2048, 8192) Y(4096, 8192) Y(4096, 16384) Y(8192, 16384)
#undef Y
        }
    }
    switch (E) {
#define X(e)                                                                                                         \
    case e: {                                                                                                        \
        if (hipError_t r = allow_lds((const void *)k_interp<R, e>, lds); r != hipSuccess)                             \
            return r;                                                                                                \
        hipLaunchKernelGGL((k_interp<R, e>), dim3((unsigned)a.batch), dim3(a.T), lds, s, (const V *)in, (V *)ws, a);  \
        return hipGetLastError();                                                                                    \
    }
        X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(15) X(16) X(20) X(24)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}
} // namespace

bool interp_width_ok(int E)
{
    switch (E) {
    case 2: case 3: case 4: case 5: case 6: case 8: case 10: case 12: case 15: case 16: case 20: case 24:
        return true;
    default:
        return false;
    }
}

hipError_t launch_interp(bool fp64, int E, const void *in, void *ws, const InterpArgs &a, size_t lds, hipStream_t s)
{
    return fp64 ? launch_interp_t<double>(E, in, ws, a, lds, s) : launch_interp_t<float>(E, in, ws, a, lds, s);
}

namespace {
template <typename R, int E, int NF1, int NF2, int LB>
hipError_t launch_fused_t(const void *in, void *out, const InterpArgs &a, size_t lds, hipStream_t s)
{
    using V = typename Vec<R>::T;
    if (a.T > LB)
        return hipErrorInvalidValue;
    auto kern = k_os_fused<R, E, NF1, NF2, LB>;
    if (hipError_t r = allow_lds((const void *)kern, lds); r != hipSuccess)
        return r;
    hipLaunchKernelGGL(kern, dim3((unsigned)a.batch), dim3(a.T), lds, s, (const V *)in, (V *)out, a);
    return hipGetLastError();
}

// (N, P N) pairs with a fused instantiation: FP32 at 16 values per thread
// (up to 1024 threads), FP64 at 16 (up to 512 threads).
#define LCT_OS_FUSED_F32(Y)                                                                                        \
    Y(float, 16, 1024, 2048, 1024) Y(float, 16, 1024, 4096, 1024) Y(float, 16, 2048, 4096, 1024)                    \
    Y(float, 16, 2048, 8192, 1024) Y(float, 16, 4096, 8192, 1024) Y(float, 16, 4096, 16384, 1024)                   \
    Y(float, 16, 8192, 16384, 1024)
#define LCT_OS_FUSED_F64(Y)                                                                                        \
    Y(double, 16, 1024, 2048, 512) Y(double, 16, 1024, 4096, 512) Y(double, 16, 2048, 4096, 512)                    \
    Y(double, 16, 2048, 8192, 512) Y(double, 16, 4096, 8192, 512)
} // namespace

int oversampled_fused_width(bool fp64, int N, int M)
{
#define Y(R, e, n, m, lb)                                                                                            \
    if (N == n && M == m)                                                                                            \
        return e;
    if (fp64) {
        LCT_OS_FUSED_F64(Y)
    } else {
        LCT_OS_FUSED_F32(Y)
    }
#undef Y
    return 0;
}

hipError_t launch_oversampled_fused(bool fp64, int E, const void *in, void *out, const InterpArgs &a, size_t lds,
                                    hipStream_t s)
{
    const int M = a.N * a.P;
    if (E != oversampled_fused_width(fp64, a.N, M) || !is_fixed_sched(a.sc1, a.N, E) ||
        !is_fixed_sched(a.sc2, M, E) || a.T != M / E)
        return hipErrorNotSupported;
#define Y(R, e, n, m, lb)                                                                                            \
    if (a.N == n && M == m)                                                                                          \
        return launch_fused_t<R, e, n, m, lb>(in, out, a, lds, s);
    if (fp64) {
        LCT_OS_FUSED_F64(Y)
    } else {
        LCT_OS_FUSED_F32(Y)
    }
#undef Y
    return hipErrorNotSupported;
}

hipError_t launch_window(bool fp64, const void *fine, void *out, int N, int M, int off, int64_t batch, hipStream_t s)
{
    if (batch <= 0)
        return hipSuccess;
    const int bs = 256;
    const dim3 grid((unsigned)((N + bs - 1) / bs), (unsigned)(batch < 65535 ? batch : 65535));
    if (fp64)
        hipLaunchKernelGGL(k_window<double>, grid, dim3(bs), 0, s, (const double2 *)fine, (double2 *)out, N, M, off,
                           batch);
    else
        hipLaunchKernelGGL(k_window<float>, grid, dim3(bs), 0, s, (const float2 *)fine, (float2 *)out, N, M, off,
                           batch);
    return hipGetLastError();
}

} // namespace lctk
