// inst_lct_f64.hip - explicit kernel instantiations (one translation unit per kind and
// precision so that they compile in parallel).
#include "kernels_impl.hpp"

namespace lctk {

hipError_t dispatch_lct_f64(int E, const void *in, void *out, const LctArgs &a, int nb, int bs, size_t lds,
                            hipStream_t s)
{
    // compile-time radix schedules (E = 16) for the common lengths; the
    // instantiations with N / 16 >= 256 threads assume one signal per
    // work-group
    if (E == 16 && is_fixed_sched(a.sc, a.N, 16) && (a.N / 16 < 256 || a.S == 1)) {
        // N = 4096: one signal of 256 threads per work-group, exchanged through
        // LDS in real and imaginary halves (34.8 KiB), so that registers, not
        // LDS, set how many work-groups share a CU
        if (a.N == 4096 && bs == 256)
            return launch_lct_t<double, 16, 4096, false, 256, true>(in, out, a, nb, bs,
                                                                    (size_t)lds_elems(4096) * sizeof(double), s);
        switch (a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_lct_t<double, 16, n>(in, out, a, nb, bs, lds, s);
            X(256) X(512) X(1024) X(2048) X(4096) X(8192)
#undef X
        default:
            break;
        }
    }
    // lengths 3 2^k (E = 12) and 5 2^k (E = 10) with their compile-time schedules
    if ((E == 12 || E == 10) && is_fixed_sched(a.sc, a.N, E) && (a.N / E < 256 || a.S == 1)) {
        switch (a.N) {
#define X(e, n)                                                                                                      \
    case n:                                                                                                          \
        if (E == e)                                                                                                  \
            return launch_lct_t<double, e, n>(in, out, a, nb, bs, lds, s);                                           \
        break;
            X(12, 1536) X(12, 3072) X(12, 6144) X(10, 2560) X(10, 5120)
#undef X
        default:
            break;
        }
    }
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_lct_t<double, e, 0>(in, out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

// The windowed forward transform (the aliasing-aware mode's fine grid): fixed
// lengths with one signal per work-group.
hipError_t dispatch_lct_window_f64(int E, const void *in, void *out, const LctArgs &a, int nb, int bs, size_t lds,
                                   hipStream_t s)
{
    if (E != 16 || !is_fixed_sched(a.sc, a.N, 16) || a.S != 1 || a.mode != MODE_FWD)
        return hipErrorNotSupported;
    switch (a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_lct_window_t<double, 16, n>(in, out, a, nb, bs, lds, s);
        X(4096) X(8192)
#undef X
    default:
        return hipErrorNotSupported;
    }
}

} // namespace lctk
