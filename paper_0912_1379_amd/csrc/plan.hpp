// plan.hpp - launch geometry of the transforms: how a length is split over
// threads, work-group slots and FFT stages, chosen by a built-in heuristic or
// by the autotuner's table; and the launches that take an explicit geometry.
#pragma once
#include <stdint.h>

#include "lct_kernels.hpp"

namespace lctk {

constexpr int64_t MAX_N = int64_t(1) << 24;
constexpr size_t LDS_BYTES = 160 * 1024;

// One-pass geometry of a length-Nfft DFT held in LDS: E values per thread,
// T = Nfft / E threads per signal, S signals per work-group, stage radices.
struct Tiling {
    int E = 0, T = 0, S = 0, block = 0;
    size_t lds = 0;
    Sched sc{};
    bool ok = false;
    bool mf = false; // radix-16 stages on the matrix cores
};

// Two-pass (four-step) geometry of a length N = N1 N2 DFT: pass 1 runs C
// length-N1 column DFTs per work-group, pass 2 RR length-N2 row DFTs.
struct FsTiling {
    int N1 = 0, N2 = 0, E1 = 0, E2 = 0, T1 = 0, T2 = 0, C = 0, RR = 0, bs1 = 0, bs2 = 0;
    size_t lds1 = 0, lds2 = 0;
    Sched sc1{}, sc2{};
    bool ok = false;
    bool mf1 = false, mf2 = false; // pass 1 / pass 2 radix-16 stages on the matrix cores
};

bool smooth235(int64_t N);
int64_t single_pass_limit(bool fp64);

// Geometry from explicit choices; `ok` only if every kernel precondition
// holds (E is an instantiated width, the radices are implemented, divide E
// and multiply to the length, the block and LDS fit).
Tiling tiling_of(int64_t Nfft, bool fp64, int E, int S, const Sched &sc, size_t extra);
FsTiling fs_of(int64_t N, bool fp64, int N1, int E1, int E2, int C, int RR, const Sched &sc1, const Sched &sc2);

// Greedy radix schedule of a length-N DFT with E values per thread (largest
// radix first, radices <= maxrad dividing E); nst = -1 if none exists.
Sched greedy_sched(int64_t N, int E, int maxrad, bool rev);

// Built-in heuristic choices.
Tiling default_tiling(int64_t Nfft, bool fp64, bool frft, size_t extra);
FsTiling default_fs(int64_t N, bool fp64, bool frft = false);

// The geometry the entry points use: the autotuner's entry for (transform
// kind, signal length, precision) when one is recorded and valid, otherwise
// the heuristic.  kind: LCT_TUNE_LCT or LCT_TUNE_FRFT.
Tiling select_tiling(int kind, int64_t N, int64_t Nfft, bool fp64, size_t extra);
FsTiling select_fs(int kind, int64_t N, int64_t Nfft, bool fp64);

// With LCT_AUTOTUNE=1 in the environment, times the candidate geometries of
// both transforms for (N, prec) on the default stream when the table has no
// entry for them (plan creation calls it; FP32 and FP64 only).  With
// LCT_TUNE_CACHE=path the table is read from that file before the first
// lookup and written back after every autotune.
void autotune_on_plan(int64_t N, int prec);

// Geometry of the split-BF16 matrix-core variant (FP32 data): N a power of
// two from 256 to 2^24; E = 16, radix-16 stages first.  One pass up to
// 16384 points, beyond that N = N1 N2 with N1 = 2^floor(log2(N) / 2); a
// pass whose length is not a multiple of 256 runs on the vector units.
Tiling mfma_tiling(int64_t N);
FsTiling mfma_fs(int64_t N);

// Enumerates the candidate geometries the autotuner times.
void tiling_candidates(int64_t Nfft, bool fp64, bool frft, Tiling *out, int *n, int cap);
void fs_candidates(int64_t Nfft, bool fp64, bool frft, FsTiling *out, int *n, int cap);

// Launches with an explicit geometry (host checks of pointers and sizes are
// the caller's).
int lct_launch(const Tiling &tl, int64_t N, bool fp64, const double *M4, const LctConst *k, int mode, const void *in,
               void *out, int64_t batch, hipStream_t s);
int fs_launch(const FsTiling &f, int64_t N, bool fp64, const double *M4, const LctConst *k, int mode, const void *in,
              void *out, int64_t batch, hipStream_t s);
// spec: when non-null (and k is given, not a z = +-1 order), the kernel's
// length-2N DFT is computed once into spec (2N complex values) and shared by
// every signal of the batch.
int frft_sp_launch(const Tiling &tl, int64_t N, bool fp64, const double *Z2, const FrConst *k, const void *in,
                   void *out, int64_t batch, hipStream_t s, void *spec = nullptr);
int frft_large_launch(const FsTiling &f, int64_t N, bool fp64, const double *Z2, const FrConst *k, const void *in,
                      void *out, int64_t batch, void *ws, hipStream_t s);
int hip_status(hipError_t e);

} // namespace lctk
