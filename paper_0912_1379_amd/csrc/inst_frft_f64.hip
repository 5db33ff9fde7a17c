// inst_frft_f64.hip - explicit kernel instantiations (one translation unit per kind and
// precision so that they compile in parallel).
#include "kernels_impl.hpp"

namespace lctk {

hipError_t dispatch_frft_f64(int E, const void *in, void *out, const FrArgs &a, int nb, int bs, size_t lds,
                             hipStream_t s)
{
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
