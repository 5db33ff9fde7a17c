// inst_fs1_f32.hip - pass-1 kernels of the two-pass (four-step) LCT.
#include "fourstep_impl.hpp"

namespace lctk {

hipError_t dispatch_fs1_f32(int E, const void *in, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    if (E == 16 && is_fixed_sched(a.sc1, a.N1, 16)) {
        switch (a.N1) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_fs1_t<float, 16, false, n>(in, out, a, nb, bs, lds, s);
            LCT_FS_FIXED_LIST(X)
#undef X
        default:
            break;
        }
    }
    if ((E == 24 || E == 20) && is_fixed_sched(a.sc1, a.N1, E)) {
        switch (a.N1) {
#define X(e, n)                                                                                                      \
    case n:                                                                                                          \
        if (E == e)                                                                                                  \
            return launch_fs1_t<float, e, false, n>(in, out, a, nb, bs, lds, s);                                                  \
        break;
            LCT_FS_FIXED3_F32(X) LCT_FS_FIXED5_F32(X)
#undef X
        default:
            break;
        }
    }
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_fs1_t<float, e>(in, out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace lctk
