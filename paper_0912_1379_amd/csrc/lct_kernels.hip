// lct_kernels.hip - precision dispatch of the single-pass kernels (the
// kernels themselves are in kernels_impl.hpp, instantiated in inst_*.hip).
#include "lct_kernels.hpp"

#include <map>
#include <mutex>
#include <utility>

namespace lctk {

hipError_t allow_lds(const void *kern, size_t lds)
{
    if (lds <= 65536)
        return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> granted;
    std::lock_guard<std::mutex> lock(mu);
    size_t &g = granted[{kern, dev}];
    if (g >= lds)
        return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
        g = lds;
    return e;
}

hipError_t launch_lct(bool fp64, int E, const void *in, void *out, const LctArgs &a, int nb, int bs, size_t lds,
                      hipStream_t s)
{
    return fp64 ? dispatch_lct_f64(E, in, out, a, nb, bs, lds, s) : dispatch_lct_f32(E, in, out, a, nb, bs, lds, s);
}

hipError_t launch_lct_window(bool fp64, int E, const void *in, void *out, const LctArgs &a, int nb, int bs,
                             size_t lds, hipStream_t s)
{
    return fp64 ? dispatch_lct_window_f64(E, in, out, a, nb, bs, lds, s)
                : dispatch_lct_window_f32(E, in, out, a, nb, bs, lds, s);
}

hipError_t launch_pgrad(bool fp64, int E, const void *f, const void *g, double *grad4, const LctArgs &a, int nb,
                        int bs, size_t lds, hipStream_t s)
{
    return fp64 ? dispatch_pgrad_f64(E, f, g, grad4, a, nb, bs, lds, s)
                : dispatch_pgrad_f32(E, f, g, grad4, a, nb, bs, lds, s);
}

hipError_t launch_frft(bool fp64, int E, const void *in, void *out, const FrArgs &a, int nb, int bs, size_t lds,
                       hipStream_t s)
{
    return fp64 ? dispatch_frft_f64(E, in, out, a, nb, bs, lds, s) : dispatch_frft_f32(E, in, out, a, nb, bs, lds, s);
}

hipError_t launch_fs1(bool fp64, int E, const void *in, void *out, const FsArgs &a, int nb, int bs, size_t lds,
                      hipStream_t s)
{
    return fp64 ? dispatch_fs1_f64(E, in, out, a, nb, bs, lds, s) : dispatch_fs1_f32(E, in, out, a, nb, bs, lds, s);
}

hipError_t launch_fs2(bool fp64, int E, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    return fp64 ? dispatch_fs2_f64(E, out, a, nb, bs, lds, s) : dispatch_fs2_f32(E, out, a, nb, bs, lds, s);
}

hipError_t launch_frl1(bool fp64, int E, const void *in, void *ws, const FrLArgs &a, int nb, int bs, size_t lds,
                       hipStream_t s)
{
    return fp64 ? dispatch_frl1_f64(E, in, ws, a, nb, bs, lds, s) : dispatch_frl1_f32(E, in, ws, a, nb, bs, lds, s);
}

hipError_t launch_frl2(bool fp64, int E, void *ws, const FrLArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    return fp64 ? dispatch_frl2_f64(E, ws, a, nb, bs, lds, s) : dispatch_frl2_f32(E, ws, a, nb, bs, lds, s);
}

hipError_t launch_frl3(bool fp64, int E, const void *ws, void *out, const FrLArgs &a, int nb, int bs, size_t lds,
                       hipStream_t s)
{
    return fp64 ? dispatch_frl3_f64(E, ws, out, a, nb, bs, lds, s) : dispatch_frl3_f32(E, ws, out, a, nb, bs, lds, s);
}

hipError_t launch_fr_special(bool fp64, const void *in, void *out, const FrLArgs &a, hipStream_t s)
{
    return fp64 ? dispatch_fr_special_f64(in, out, a, s) : dispatch_fr_special_f32(in, out, a, s);
}

} // namespace lctk
