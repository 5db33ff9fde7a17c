// inst_fs2_f32.hip - pass-2 kernels of the two-pass (four-step) LCT.
#include "fourstep_impl.hpp"

namespace lctk {

hipError_t dispatch_fs2_f32(int E, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_fs2_t<float, e>(out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace lctk
