// inst_pgrad_f64.hip - explicit kernel instantiations (one translation unit per kind and
// precision so that they compile in parallel).
#include "kernels_impl.hpp"

namespace lctk {

hipError_t dispatch_pgrad_f64(int E, const void *f, const void *g, double *grad4, const LctArgs &a, int nb,
                              int bs, size_t lds, hipStream_t s)
{
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
