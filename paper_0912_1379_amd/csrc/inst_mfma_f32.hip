// inst_mfma_f32.hip - FP32 kernels whose radix-16 stages run on the matrix
// cores (split-BF16 products with FP32 accumulation).
#include "fourstep_impl.hpp"
#include "mfma_lct_impl.hpp"

namespace lctk {

hipError_t launch_lct_mf(const void *in, void *out, const LctArgs &a, int nblocks, int block, size_t lds,
                         hipStream_t s)
{
    // N = 4096 = 16^3: every stage on the matrix cores, HBM in and out of
    // the first and last stage directly
    if (a.N == 4096 && a.S == 1 && block == 256)
        return launch_lct_mf4096_t(in, out, a, nblocks, lds, s);
    // a 256-thread bound leaves the register file to the one work-group size
    // of N <= 4096 (no spills); larger N need up to 1024 threads
    if (block <= 256)
        return launch_lct_t<float, 16, 0, true, 256>(in, out, a, nblocks, block, lds, s);
    return launch_lct_t<float, 16, 0, true>(in, out, a, nblocks, block, lds, s);
}

// The four-step passes run 256-thread work-groups (16 lengths' worth of
// threads); the 256-thread bound leaves them the register file.
hipError_t launch_fs1_mf(const void *in, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    if (bs <= 256)
        return launch_fs1_t<float, 16, true, 0, 256>(in, out, a, nb, bs, lds, s);
    return launch_fs1_t<float, 16, true>(in, out, a, nb, bs, lds, s);
}

hipError_t launch_fs2_mf(void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s)
{
    if (bs <= 256)
        return launch_fs2_t<float, 16, true, 0, 256>(out, a, nb, bs, lds, s);
    return launch_fs2_t<float, 16, true>(out, a, nb, bs, lds, s);
}

} // namespace lctk
