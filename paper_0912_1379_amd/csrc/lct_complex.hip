// lct_complex.hip - launches of the complex-matrix LCT at the Algorithm's
// complex output nodes (cx_impl.hpp).
#include "cx_impl.hpp"

namespace lctk {

namespace {
template <typename R, int E, int NFIX = 0, int LB = max_block(sizeof(R) == 8, E), bool HX = false>
hipError_t launch_one(const void *in, void *out, const CxArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    using V = typename Vec<R>::T;
    auto kern = k_lct_cx<R, E, NFIX, LB, HX>;
    if (hipError_t r = allow_lds((const void *)kern, lds); r != hipSuccess)
        return r;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, s, (const V *)in, (V *)out, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_cx_t(int E, const void *in, void *out, const CxArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    // compile-time schedules for the common lengths (as the real-matrix LCT);
    // the instantiations with N / 16 >= 256 threads take one signal per work-group
    if (E == 16 && is_fixed_sched(a.sc, a.N, 16) && (a.N / 16 < 256 || a.S == 1)) {
        if constexpr (sizeof(R) == 8) {
            if (a.N == 4096 && bs == 256)
                return launch_one<double, 16, 4096, 256, true>(in, out, a, nb, bs,
                                                               (size_t)lds_elems(4096) * sizeof(double), s);
        }
        switch (a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_one<R, 16, n>(in, out, a, nb, bs, lds, s);
            X(256) X(512) X(1024) X(2048) X(4096) X(8192)
#undef X
        case 16384:
            if constexpr (sizeof(R) == 4)
                return launch_one<R, 16, 16384>(in, out, a, nb, bs, lds, s);
            break;
        default:
            break;
        }
    }
    // lengths 3 2^k and 5 2^k at the widths the planner gives them (FP32 24 / 20,
    // FP64 12 / 10)
    constexpr int E3 = sizeof(R) == 8 ? 12 : 24, E5 = sizeof(R) == 8 ? 10 : 20;
    if ((E == E3 || E == E5) && is_fixed_sched(a.sc, a.N, E) && (a.N / E < 256 || a.S == 1)) {
        switch (a.N) {
#define X(e, n)                                                                                                      \
    case n:                                                                                                          \
        if (E == e)                                                                                                  \
            return launch_one<R, e, n>(in, out, a, nb, bs, lds, s);                                                  \
        break;
            X(E3, 1536) X(E3, 3072) X(E3, 6144) X(E5, 2560) X(E5, 5120)
#undef X
        case 12288:
            if constexpr (sizeof(R) == 4)
                if (E == E3)
                    return launch_one<R, E3, 12288>(in, out, a, nb, bs, lds, s);
            break;
        case 10240:
            if constexpr (sizeof(R) == 4)
                if (E == E5)
                    return launch_one<R, E5, 10240>(in, out, a, nb, bs, lds, s);
            break;
        default:
            break;
        }
    }
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_one<R, e>(in, out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}
} // namespace

hipError_t launch_cx(bool fp64, int E, const void *in, void *out, const CxArgs &a, int nb, int bs, size_t lds,
                     hipStream_t s)
{
    return fp64 ? launch_cx_t<double>(E, in, out, a, nb, bs, lds, s) : launch_cx_t<float>(E, in, out, a, nb, bs, lds, s);
}

} // namespace lctk
