// inst_frft_f64.hip - explicit kernel instantiations (one translation unit per kind and
// precision so that they compile in parallel).
#include "kernels_impl.hpp"

namespace lctk {

hipError_t dispatch_frft_f64(int E, const void *in, void *out, const FrArgs &a, int nb, int bs, size_t lds,
                             hipStream_t s)
{
    // compile-time radix schedules (E = 16) for the common convolution lengths
    if (E == 16 && is_fixed_sched(a.sc, 2 * a.N, 16)) {
        switch (2 * a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        if (bs <= tight_bound(n))                                                                                    \
            return launch_frft_t<double, 16, n, tight_bound(n)>(in, out, a, nb, bs, lds, s);                          \
        return launch_frft_t<double, 16, n>(in, out, a, nb, bs, lds, s);
            X(512) X(1024) X(2048) X(4096) X(8192)
#undef X
        default:
            break;
        }
    }
    // E = 8 (the tuner's alternative to the default 16)
    if (E == 8 && is_fixed_sched(a.sc, 2 * a.N, 8)) {
        switch (2 * a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_frft_t<double, 8, n>(in, out, a, nb, bs, lds, s);
            X(2048) X(4096) X(8192)
#undef X
        default:
            break;
        }
    }
    // convolution lengths 3 2^k at E = 12 (the kernel's spectrum held in
    // registers in every spectrum mode, 234-248 VGPRs, no spills)
    if (E == 12 && is_fixed_sched(a.sc, 2 * a.N, 12)) {
        switch (2 * a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_frft_t<double, 12, n>(in, out, a, nb, bs, lds, s);
            X(3072) X(6144)
#undef X
        default:
            break;
        }
    }
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_frft_t<double, e>(in, out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace lctk
