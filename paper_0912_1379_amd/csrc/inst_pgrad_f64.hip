// inst_pgrad_f64.hip - explicit kernel instantiations (one translation unit per kind and
// precision so that they compile in parallel).
#include "kernels_impl.hpp"

namespace lctk {

hipError_t dispatch_pgrad_f64(int E, const void *f, const void *g, double *grad4, const LctArgs &a, int nb,
                              int bs, size_t lds, hipStream_t s)
{
    // compile-time radix schedules (E = 16) for the common lengths
    if (E == 16 && is_fixed_sched(a.sc, a.N, 16)) {
        switch (a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        if (bs <= tight_bound(n))                                                                                    \
            return launch_pgrad_t<double, 16, n, tight_bound(n)>(f, g, grad4, a, nb, bs, lds, s);                     \
        return launch_pgrad_t<double, 16, n>(f, g, grad4, a, nb, bs, lds, s);
            X(256) X(512) X(1024) X(2048) X(4096) X(8192)
#undef X
        default:
            break;
        }
    }
    // lengths 3 2^k and 5 2^k at the planner's widths, work-groups of up to 256
    // threads (their compile-time schedules fit that bound's registers with few
    // or no spills; the runtime-schedule kernel spills 300 VGPRs and more)
    if ((E == 12 || E == 10) && bs <= 256 && is_fixed_sched(a.sc, a.N, E)) {
        switch (a.N) {
#define X(e, n)                                                                                                      \
    case n:                                                                                                          \
        if (E == e)                                                                                                  \
            return launch_pgrad_t<double, e, n, 256>(f, g, grad4, a, nb, bs, lds, s);                                  \
        break;
            X(12, 1536) X(12, 3072) X(10, 2560)
#undef X
        default:
            break;
        }
    }
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_pgrad_t<double, e>(f, g, grad4, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace lctk
