// lct_complex.hip - launches of the complex-matrix LCT at the Algorithm's
// complex output nodes (cx_impl.hpp).
#include "cx_impl.hpp"

namespace lctk {

namespace {
template <typename R>
hipError_t launch_cx_t(int E, const void *in, void *out, const CxArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    using V = typename Vec<R>::T;
    switch (E) {
#define X(e)                                                                                                         \
    case e: {                                                                                                        \
        if (hipError_t r = allow_lds((const void *)k_lct_cx<R, e>, lds); r != hipSuccess)                             \
            return r;                                                                                                \
        hipLaunchKernelGGL((k_lct_cx<R, e>), dim3(nb), dim3(bs), lds, s, (const V *)in, (V *)out, a);                 \
        return hipGetLastError();                                                                                    \
    }
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}
} // namespace

hipError_t launch_cx(bool fp64, int E, const void *in, void *out, const CxArgs &a, int nb, int bs, size_t lds,
                     hipStream_t s)
{
    return fp64 ? launch_cx_t<double>(E, in, out, a, nb, bs, lds, s) : launch_cx_t<float>(E, in, out, a, nb, bs, lds, s);
}

} // namespace lctk
