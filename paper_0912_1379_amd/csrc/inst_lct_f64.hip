// inst_lct_f64.hip - explicit kernel instantiations (one translation unit per kind and
// precision so that they compile in parallel).
#include "kernels_impl.hpp"

namespace lctk {

hipError_t dispatch_lct_f64(int E, const void *in, void *out, const LctArgs &a, int nb, int bs, size_t lds,
                            hipStream_t s)
{
    // compile-time schedule for the geometry E=16 S=1 rad=16.16.16 of N = 4096
    // (that kernel assumes one signal per work-group)
    if (a.N == 4096 && E == 16 && a.S == 1 && a.sc.nst == 3 && a.sc.rad[0] == 16 && a.sc.rad[1] == 16 && a.sc.rad[2] == 16)
        return launch_lct_t<double, 16, 4096>(in, out, a, nb, bs, lds, s);
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

} // namespace lctk
