// inst_fs2_f64.hip - pass-2 kernels of the two-pass (four-step) LCT.
#include "fourstep_impl.hpp"

namespace lctk {

hipError_t dispatch_fs2_f64(int E, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    if (E == 16 && is_fixed_sched(a.sc2, a.N2, 16)) {
        switch (a.N2) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_fs2_t<double, 16, false, n>(out, a, nb, bs, lds, s);
            LCT_FS_FIXED_LIST(X)
#undef X
        default:
            break;
        }
    }
    if ((E == 12 || E == 10) && is_fixed_sched(a.sc2, a.N2, E)) {
        switch (a.N2) {
#define X(e, n)                                                                                                      \
    case n:                                                                                                          \
        if (E == e)                                                                                                  \
            return launch_fs2_t<double, e, false, n>(out, a, nb, bs, lds, s);                                                  \
        break;
            LCT_FS_FIXED3_F64(X) LCT_FS_FIXED5_F64(X)
#undef X
        default:
            break;
        }
    }
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_fs2_t<double, e>(out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace lctk
