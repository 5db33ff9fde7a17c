// inst_fs1_f64.hip - pass-1 kernels of the two-pass (four-step) LCT.
#include "fourstep_impl.hpp"

namespace lctk {

hipError_t dispatch_fs1_f64(int E, const void *in, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_fs1_t<double, e>(in, out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace lctk
