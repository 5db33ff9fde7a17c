// inst_frl_f64.hip - kernels of the fractional transform beyond one work-group's LDS.
#include "frft_large_impl.hpp"

namespace lctk {

hipError_t dispatch_frl1_f64(int E, const void *in, void *ws, const FrLArgs &a, int nb, int bs, size_t lds,
                               hipStream_t s)
{
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_frl1_t<double, e>(in, ws, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t dispatch_frl2_f64(int E, void *ws, const FrLArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_frl2_t<double, e>(ws, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t dispatch_frl3_f64(int E, const void *ws, void *out, const FrLArgs &a, int nb, int bs, size_t lds,
                               hipStream_t s)
{
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_frl3_t<double, e>(ws, out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t dispatch_fr_special_f64(const void *in, void *out, const FrLArgs &a, hipStream_t s)
{
    return launch_fr_special_t<double>(in, out, a, s);
}

} // namespace lctk
