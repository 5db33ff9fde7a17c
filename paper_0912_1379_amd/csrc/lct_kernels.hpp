// lct_kernels.hpp - kernel argument blocks and launch entry points shared by
// the host API (lct_api.hip) and the kernels (lct_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"
#include "lct_params.hpp"

namespace lctk {

// Raises `kern`'s dynamic LDS limit on the current device to at least `lds`
// bytes when `lds` exceeds the 64 KiB default.  The attribute persists, so it
// is set once per (kernel, device) and later calls only look it up: setting
// it on every launch puts a host round trip between back-to-back launches.
hipError_t allow_lds(const void *kern, size_t lds);

struct LctArgs {
    int N;          // signal length
    int T;          // threads per signal (N / E)
    int S;          // signals per work-group
    int mode;       // 0 forward, 1 adjoint
    int64_t batch;  // number of signals
    const double *M4; // per-signal (a, b, c, d) on the device, or null
    LctConst k;     // constants when M4 is null
    NConst nc;      // N-only constants (per-signal constants derive from them)
    Sched sc;       // radix schedule of the length-N DFT
    int win_off;    // windowed instantiations: output positions [win_off, win_off + win_n)
    int win_n;      //   of each signal, stored contiguously (win_n per signal)
};

// Kernel-spectrum modes of the single-pass fractional transform.
enum { SPEC_NONE = 0, SPEC_WRITE = 1, SPEC_READ = 2 };

struct FrArgs {
    int N;          // signal length (the convolution length is 2N)
    int T;          // threads per signal (2N / E)
    int S;          // signals per work-group
    int spec_mode;  // SPEC_NONE: every signal transforms the kernel itself;
                    // SPEC_WRITE: one work-group stores the kernel's DFT to `spec`;
                    // SPEC_READ: every signal loads it from `spec` (one shared order)
    int64_t batch;
    const double *Z2; // per-signal (re z, im z) on the device, or null
    FrConst k;        // constants when Z2 is null
    Sched sc;         // radix schedule of the length-2N DFT
    void *spec;       // 2N complex values in natural order (SPEC_WRITE / SPEC_READ)
};

struct FsArgs {
    int N, N1, N2;  // N = N1 N2
    int C;          // columns per pass-1 work-group
    int RR;         // rows per pass-2 work-group
    int T1, T2;     // threads per length-N1 / length-N2 DFT
    int mode;       // 0 forward, 1 adjoint
    int64_t batch;
    const double *M4;
    LctConst k;
    NConst nc;
    Sched sc1, sc2;
};

// Values per thread (E) with instantiated kernels.
#define LCT_E_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(9) X(10) X(12) X(15) X(16) X(18) X(20) X(24) X(25) X(27) X(30)

// Largest work-group a kernel instantiation accepts (its launch bound): the
// register budget per thread is 512 / (waves per SIMD) VGPRs, so larger E
// (more values per thread) gets a smaller bound.
__host__ __device__ constexpr int max_block(bool fp64, int E)
{
    return fp64 ? (E <= 8 ? 1024 : 512) : (E <= 16 ? 1024 : 512);
}

hipError_t launch_lct(bool fp64, int E, const void *in, void *out, const LctArgs &a, int nblocks, int block,
                      size_t lds, hipStream_t s);
// Forward transform storing only a.win_n outputs from position a.win_off per
// signal (fixed lengths with one signal per work-group); hipErrorNotSupported
// where no such instantiation exists.
hipError_t launch_lct_window(bool fp64, int E, const void *in, void *out, const LctArgs &a, int nblocks, int block,
                             size_t lds, hipStream_t s);
hipError_t launch_pgrad(bool fp64, int E, const void *f, const void *g, double *grad4, const LctArgs &a,
                        int nblocks, int block, size_t lds, hipStream_t s);
hipError_t launch_frft(bool fp64, int E, const void *in, void *out, const FrArgs &a, int nblocks, int block,
                       size_t lds, hipStream_t s);

#define LCTK_DISPATCH_DECL(tag)                                                                                    \
    hipError_t dispatch_lct_##tag(int E, const void *in, void *out, const LctArgs &a, int nb, int bs, size_t lds,    \
                                  hipStream_t s);                                                                    \
    hipError_t dispatch_frft_##tag(int E, const void *in, void *out, const FrArgs &a, int nb, int bs, size_t lds,    \
                                   hipStream_t s);                                                                   \
    hipError_t dispatch_pgrad_##tag(int E, const void *f, const void *g, double *grad4, const LctArgs &a, int nb,    \
                                    int bs, size_t lds, hipStream_t s);                                              \
    hipError_t dispatch_lct_window_##tag(int E, const void *in, void *out, const LctArgs &a, int nb, int bs,         \
                                         size_t lds, hipStream_t s);
// Fractional transform beyond one work-group: length L = 2N = L1 L2.
struct FrLArgs {
    int N, L, L1, L2;
    int C, RR, T1, T2;
    int64_t batch;
    const double *Z2;
    FrConst k;
    Sched sc1, sc2;
    int spec_mode; // pass 2: SPEC_NONE, or one order for the batch (SPEC_WRITE once, then SPEC_READ)
};
// FP32 with the radix-16 stages on the matrix cores (E = 16 only).
hipError_t launch_lct_mf(const void *in, void *out, const LctArgs &a, int nblocks, int block, size_t lds,
                         hipStream_t s);
hipError_t launch_fs1_mf(const void *in, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s);
hipError_t launch_fs2_mf(void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s);
hipError_t launch_frl1(bool fp64, int E, const void *in, void *ws, const FrLArgs &a, int nb, int bs, size_t lds,
                       hipStream_t s);
hipError_t launch_frl2(bool fp64, int E, void *ws, const FrLArgs &a, int nb, int bs, size_t lds, hipStream_t s);
hipError_t launch_frl3(bool fp64, int E, const void *ws, void *out, const FrLArgs &a, int nb, int bs, size_t lds,
                       hipStream_t s);
hipError_t launch_fr_special(bool fp64, const void *in, void *out, const FrLArgs &a, hipStream_t s);
#define LCTK_FRL_DECL(tag)                                                                                         \
    hipError_t dispatch_frl1_##tag(int E, const void *in, void *ws, const FrLArgs &a, int nb, int bs, size_t lds,  \
                                   hipStream_t s);                                                                \
    hipError_t dispatch_frl2_##tag(int E, void *ws, const FrLArgs &a, int nb, int bs, size_t lds, hipStream_t s);  \
    hipError_t dispatch_frl3_##tag(int E, const void *ws, void *out, const FrLArgs &a, int nb, int bs, size_t lds, \
                                   hipStream_t s);                                                                \
    hipError_t dispatch_fr_special_##tag(const void *in, void *out, const FrLArgs &a, hipStream_t s);
LCTK_FRL_DECL(f32)
LCTK_FRL_DECL(f64)
#undef LCTK_FRL_DECL
hipError_t launch_fs1(bool fp64, int E, const void *in, void *out, const FsArgs &a, int nb, int bs, size_t lds,
                      hipStream_t s);
hipError_t launch_fs2(bool fp64, int E, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s);
#define LCTK_FS_DECL(tag)                                                                                          \
    hipError_t dispatch_fs1_##tag(int E, const void *in, void *out, const FsArgs &a, int nb, int bs, size_t lds,     \
                                  hipStream_t s);                                                                  \
    hipError_t dispatch_fs2_##tag(int E, void *out, const FsArgs &a, int nb, int bs, size_t lds, hipStream_t s);
LCTK_FS_DECL(f32)
LCTK_FS_DECL(f64)
#undef LCTK_FS_DECL
LCTK_DISPATCH_DECL(f32)
LCTK_DISPATCH_DECL(f64)
#undef LCTK_DISPATCH_DECL

// Aliasing-aware LCT: trigonometric interpolation onto the grid P times finer
// (one work-group of T = P N / E threads per signal) and the window copy.
struct InterpArgs {
    int N, P;       // samples, oversampling factor (fine length P N)
    int T;          // threads per work-group: P N / E
    int T1;         // threads of the length-N DFT: N / E (<= T)
    int64_t batch;
    Sched sc1, sc2; // schedules of the length-N and length-P N DFTs
    LctConst k;     // fused launch: the fine-grid transform's constants
};
bool interp_width_ok(int E);
// The interpolation, the fine-grid transform and the window in one kernel
// (compile-time schedules for the common (N, P N) pairs at E = 16: FP32 up to
// P N = 16384, FP64 up to 8192); hipErrorNotSupported elsewhere.
// oversampled_fused_width: the E of the fused instantiation for (N, M = P N),
// 0 if there is none.
int oversampled_fused_width(bool fp64, int N, int M);
hipError_t launch_oversampled_fused(bool fp64, int E, const void *in, void *out, const InterpArgs &a, size_t lds,
                                    hipStream_t s);

// LCT of a complex matrix at the Algorithm's complex output nodes: per-n^2
// log-modulus and turns (double-double) of the pre- and post-diagonals, and
// the amplitude.
struct CxConst {
    double pre_mag, pre_hi, pre_lo;
    double post_mag, post_hi, post_lo;
    double amp_re, amp_im;
};
struct CxArgs {
    int N, T, S;
    int64_t batch;
    CxConst k;
    Sched sc;
};
hipError_t launch_cx(bool fp64, int E, const void *in, void *out, const CxArgs &a, int nb, int bs, size_t lds,
                     hipStream_t s);
hipError_t launch_interp(bool fp64, int E, const void *in, void *ws, const InterpArgs &a, size_t lds, hipStream_t s);
hipError_t launch_window(bool fp64, const void *fine, void *out, int N, int M, int off, int64_t batch, hipStream_t s);

} // namespace lctk
