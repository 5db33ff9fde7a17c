// inst_frft_f32.hip - explicit kernel instantiations (one translation unit per kind and
// precision so that they compile in parallel).
#include "kernels_impl.hpp"

namespace lctk {

namespace {
template <int L>
hipError_t launch_frft24(const void *in, void *out, const FrArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    auto kern = k_frft<float, 24, L>;
    if (hipError_t e = allow_lds((const void *)kern, lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), lds, s, (const float2 *)in, (float2 *)out, a);
    return hipGetLastError();
}
} // namespace

hipError_t dispatch_frft_f32(int E, const void *in, void *out, const FrArgs &a, int nb, int bs, size_t lds,
                             hipStream_t s)
{
    // compile-time radix schedules (E = 16) for the common convolution lengths
    if (E == 16 && is_fixed_sched(a.sc, 2 * a.N, 16)) {
        switch (2 * a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        if (bs <= tight_bound(n))                                                                                    \
            return launch_frft_t<float, 16, n, tight_bound(n)>(in, out, a, nb, bs, lds, s);                          \
        return launch_frft_t<float, 16, n>(in, out, a, nb, bs, lds, s);
            X(512) X(1024) X(2048) X(4096) X(8192) X(16384)
#undef X
        default:
            break;
        }
    }
    // convolution lengths 3 2^k at E = 24, every spectrum mode through the
    // instantiation that holds the kernel's spectrum in registers (the one that
    // reads a shared spectrum at the product spills at E = 24; at E = 20, for
    // 5 2^k, every compile-time form spills where the runtime one does not)
    if (E == 24 && is_fixed_sched(a.sc, 2 * a.N, 24)) {
        switch (2 * a.N) {
#define X(n)                                                                                                         \
    case n:                                                                                                          \
        return launch_frft24<n>(in, out, a, nb, bs, lds, s);
            X(3072) X(6144) X(12288)
#undef X
        default:
            break;
        }
    }
    switch (E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        return launch_frft_t<float, e>(in, out, a, nb, bs, lds, s);
        LCT_E_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace lctk
