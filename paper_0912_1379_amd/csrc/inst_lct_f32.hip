// inst_lct_f32.hip - explicit kernel instantiations (one translation unit per kind and
// precision so that they compile in parallel).
#include "kernels_impl.hpp"

namespace lctk {

hipError_t dispatch_lct_f32(int E, const void *in, void *out, const LctArgs &a, int nb, int bs, size_t lds,
                            hipStream_t s)
{
    // compile-time radix schedules (E = 16) for the common lengths; the
    // instantiations with N / 16 >= 256 threads assume one signal per
    // work-group
    if (E == 16 && is_fixed_sched(a.sc, a.N, 16) && (a.N / 16 < 256 || a.S == 1)) {
        switch (a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_lct_t<float, 16, n>(in, out, a, nb, bs, lds, s);
            X(256) X(512) X(1024) X(2048) X(4096) X(8192) X(16384)
#undef X
        default:
            break;
        }
    }
    // lengths 3 2^k (E = 24) and 5 2^k (E = 20) with their compile-time schedules
    if ((E == 24 || E == 20) && is_fixed_sched(a.sc, a.N, E) && (a.N / E < 256 || a.S == 1)) {
        switch (a.N) {
#define X(e, n)                                                                                                      \
    case n:                                                                                                          \
        if (E == e)                                                                                                  \
            return launch_lct_t<float, e, n>(in, out, a, nb, bs, lds, s);                                            \
        break;
            X(24, 1536) X(24, 3072) X(24, 6144) X(24, 12288) X(20, 2560) X(20, 5120) X(20, 10240)
#undef X
        default:
            break;
        }
    }
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_lct_t<float, e, 0>(in, out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

// The windowed forward transform (the aliasing-aware mode's fine grid): fixed
// lengths with one signal per work-group.
hipError_t dispatch_lct_window_f32(int E, const void *in, void *out, const LctArgs &a, int nb, int bs, size_t lds,
                                   hipStream_t s)
{
    if (E != 16 || !is_fixed_sched(a.sc, a.N, 16) || a.S != 1 || a.mode != MODE_FWD)
        return hipErrorNotSupported;
    switch (a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_lct_window_t<float, 16, n>(in, out, a, nb, bs, lds, s);
        X(4096) X(8192) X(16384)
#undef X
    default:
        return hipErrorNotSupported;
    }
}

} // namespace lctk
