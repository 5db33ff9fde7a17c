// ragged_impl.hpp - one persistent launch over a ragged batch: signals of
// different lengths, each an LCT (one matrix per signal) or a same-grid
// fractional transform (one order per signal).
//
// The host groups the signals into work items and sorts them by estimated
// cost, largest first (LPT).  Every work-group of 256 threads takes the next
// item from a device counter until the list is exhausted; an item never waits
// for another item, so every work-group finishes.  Each item kind is a
// separate (not inlined) function so that each gets its own register
// allocation inside the one kernel.
//   RI_LCT_GROUP   S signals of one length N <= 6144 (one slot each, in LDS)
//   RI_FRFT_GROUP  S signals of one length with 2N <= 6144
//   RI_LCT_BIG     one signal, four-step inside the work-group: column tiles
//                  (pre-chirp, DFT, twiddle, transposed store to out), then
//                  row tiles (DFT, post-chirp, store in place)
//   RI_FRFT_BIG    one signal, the length-2N convolution through the
//                  signal's workspace region (two spectra): column passes of
//                  the data and of the kernel, one row pass that finishes both
//                  spectra, multiplies them and starts the inverse transform,
//                  and a closing column pass that writes the outputs
#pragma once
#include "frft_large_impl.hpp"

namespace lctk {

constexpr int RAG_THREADS = 256;

enum RagKind { RI_LCT_GROUP = 0, RI_FRFT_GROUP = 1, RI_LCT_BIG = 2, RI_FRFT_BIG = 3 };

// A descriptor as the C ABI defines it (lct_desc).
struct RagDesc {
    int64_t offset;
    int32_t N;
    int32_t kind;
    int32_t prec;
    int32_t pad;
    double p[4];
};

struct RagSize {
    int N;
    int E, T, S;          // single pass: values per thread, threads per signal, slots
    int N1, N2, E1, E2;   // four-step split of the DFT length (N or 2N)
    int T1, T2, C, RR;
    NConst nc;
    Sched sc, sc1, sc2;
};

struct RagItem {
    int kind;
    int size;   // index into the size table
    int first;  // first entry in the signal list
    int count;  // signals in this item
};

struct RagArgs {
    const RagDesc *desc;
    const int *sig;
    const RagItem *items;
    const RagSize *sizes;
    const int64_t *wsoff; // per signal: element offset of its workspace region (big fractional transforms)
    int nitems;
    int *head;
    const float2 *in;
    float2 *out;
    float2 *ws;
};

using CF = C<float>;

// --- one-pass LCT of up to S signals of length N ---------------------------
template <int E>
__device__ __noinline__ void rag_lct_group(const RagArgs &a, const RagItem &it, const RagSize &z, CF *smem)
{
    const int N = z.N, T = z.T;
    const int tid = (int)threadIdx.x;
    const int sl = tid / T, t = tid - sl * T;
    const bool live = sl < it.count;
    const int s = live ? a.sig[it.first + sl] : a.sig[it.first];
    const RagDesc d = a.desc[s];
    const float2 *src = a.in + d.offset;
    float2 *dst = a.out + d.offset;
    const double inv2N = 0.5 / (double)N;
    CF v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = live ? ldc<float>(src + t + T * e) : CF{0.f, 0.f};
    const LctConst k = lct_const_from(z.nc, d.p[0], d.p[1], d.p[2], d.p[3]);
    const float mag = (float)k.amp_mag;
    if (k.b0) {
        const ThreadChirp cb = thread_chirp(k.post_hi, k.post_lo, false, t, T, N, inv2N, k.amp_turns);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (live)
                stc<float>(dst + t + T * e, cmul(v[e], cscale(chirp_at<float>(cb, e), mag)));
            v[e] = CF{0.f, 0.f};
        }
    } else {
        const ThreadChirp c = thread_chirp(k.pre_hi, k.pre_lo, true, t, T, N, inv2N);
#pragma unroll
        for (int e = 0; e < E; ++e)
            v[e] = cmul(v[e], chirp_at<float>(c, e));
    }
    fft_lds<E>(v, smem + (size_t)sl * lds_elems(N), t, T, z.sc);
    if (live && !k.b0) {
        const ThreadChirp c = thread_chirp(k.post_hi, k.post_lo, true, t, T, N, inv2N, k.amp_turns);
#pragma unroll
        for (int e = 0; e < E; ++e)
            stc<float>(dst + t + T * e, cscale(cmul(v[e], chirp_at<float>(c, e)), mag));
    }
}

// --- one-pass fractional transform of up to S signals (length-2N convolution)
template <int E>
__device__ __noinline__ void rag_frft_group(const RagArgs &a, const RagItem &it, const RagSize &z, CF *smem)
{
    const int N = z.N, L = 2 * N, T = z.T;
    const int tid = (int)threadIdx.x;
    const int sl = tid / T, t = tid - sl * T;
    const bool live = sl < it.count;
    const int s = live ? a.sig[it.first + sl] : a.sig[it.first];
    const RagDesc d = a.desc[s];
    const float2 *src = a.in + d.offset;
    float2 *dst = a.out + d.offset;
    const FrConst k = fr_const(N, d.p[0], d.p[1], false);
    CF *lds = smem + (size_t)sl * lds_elems(L);
    if (k.special) {
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int j = t + T * e;
            if (live)
                stc<float>(dst + j, cscale(ldc<float>(src + (k.special == 1 ? j : N - 1 - j)), (float)k.cre));
        }
    }
    // kernel at m = p = t + T e up to N, m = L - p = (L - t) - T e beyond;
    // data chirp at n_p = 2p - N + 1 = (2t - N + 1) + 2T e (E is even)
    CF K[E];
    {
        const GaussPoly lo = gauss_poly(k.kmag, k.kph_hi, k.kph_lo, t, T);
        const GaussPoly hi = gauss_poly(k.kmag, k.kph_hi, k.kph_lo, L - t, -T);
#pragma unroll
        for (int e = 0; e < E; ++e)
            K[e] = t + T * e <= N ? gauss_at(lo, e) : gauss_at(hi, e);
    }
    fft_lds<E>(K, lds, t, T, z.sc);
    const GaussPoly dch = gauss_poly(k.dmag, k.dph_hi, k.dph_lo, 2 * t - N + 1, 2 * T);
    CF v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = t + T * e;
        CF x = {0.f, 0.f};
        if (e < E / 2 && live && !k.special)
            x = cmul(ldc<float>(src + (k.hankel ? N - 1 - p : p)), gauss_at(dch, e));
        v[e] = x;
    }
    fft_lds<E>(v, lds, t, T, z.sc);
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = cconj(cmul(v[e], K[e]));
    fft_lds<E>(v, lds, t, T, z.sc);
    if (live && !k.special) {
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int j = t + T * e;
            CF y = cmul(cconj(v[e]), gauss_at(dch, e));
            stc<float>(dst + j, cmul(y, CF{(float)k.cre, (float)k.cim}));
        }
    }
}

// --- four-step building blocks inside one work-group --------------------------
// Column pass over a length-M = N1 N2 sequence: for every tile of C columns,
// elements i = n1 N2 + n2 come from `load(i, e)` after `load.begin(t, n2)`
// (per-thread set-up for the positions (t + T1 e) N2 + n2); after the
// length-N1 DFT and the twiddle W_M^(n2 k1) the tile is stored transposed:
// dst[n2 N1 + k1].
template <int E1, class Load>
__device__ __forceinline__ void rag_cols(const RagSize &z, int M, CF *smem, float2 *dst, Load load)
{
    const int N1 = z.N1, N2 = z.N2, Cc = z.C, T1 = z.T1;
    const int tid = (int)threadIdx.x;
    const int sl = tid % Cc, t = tid / Cc;
    const int sl2 = tid / T1, t2 = tid - sl2 * T1;
    CF *lds = smem + (size_t)sl * lds_elems(N1);
    const CF *l2 = smem + (size_t)sl2 * lds_elems(N1);
    for (int n20 = 0; n20 < N2; n20 += Cc) {
        // a last, partial tile leaves its excess column slots idle (zeros)
        const int n2 = n20 + sl;
        const bool colok = n2 < N2;
        CF v[E1];
        load.begin(t, n2);
#pragma unroll
        for (int e = 0; e < E1; ++e)
            v[e] = colok ? load((t + T1 * e) * N2 + n2, e) : CF{0.f, 0.f};
        fft_lds<E1>(v, lds, t, T1, z.sc1);
        const double A = -(double)umod24(n2 * t, M) / (double)M;
        const double B = -(double)umod24(n2 * T1, M) / (double)M;
#pragma unroll
        for (int e = 0; e < E1; ++e)
            v[e] = cmul(v[e], cis_turns_from<float>(frac_turns(fma(B, (double)e, A))));
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E1; ++e)
            lds[lds_pad(t + T1 * e)] = v[e];
        __syncthreads();
        if (n20 + sl2 < N2) {
#pragma unroll
            for (int e = 0; e < E1; ++e)
                stc<float>(dst + (size_t)(n20 + sl2) * N1 + t2 + T1 * e, l2[lds_pad(t2 + T1 * e)]);
        }
    }
    __syncthreads(); // the work-group's stores are visible to its next loads
}

// Row pass: for every tile of RR rows k1, the length-N2 DFT over n2 of
// src[n2 N1 + k1]; after `store.begin(k1, t)`, `store(k1, k2, value, e)`
// receives DFT index k1 + N1 k2 (k2 = t + T2 e, stored at k2 N1 + k1).
template <int E2, class Store>
__device__ __forceinline__ void rag_rows(const RagSize &z, CF *smem, const float2 *src, Store store)
{
    const int N1 = z.N1, RR = z.RR, T2 = z.T2;
    const int tid = (int)threadIdx.x;
    const int r = tid % RR, t = tid / RR;
    CF *lds = smem + (size_t)r * lds_elems(z.N2);
    for (int k10 = 0; k10 < N1; k10 += RR) {
        // a last, partial tile leaves its excess row slots idle
        const int k1 = k10 + r;
        const bool rowok = k1 < N1;
        CF v[E2];
#pragma unroll
        for (int e = 0; e < E2; ++e)
            v[e] = rowok ? ldc<float>(src + (size_t)(t + T2 * e) * N1 + k1) : CF{0.f, 0.f};
        fft_lds<E2>(v, lds, t, T2, z.sc2);
        if (rowok) {
            store.begin(k1, t);
#pragma unroll
            for (int e = 0; e < E2; ++e)
                store(k1, t + T2 * e, v[e], e);
        }
    }
    __syncthreads();
}

// Convolution row pass of the fractional transform: for every tile of RR
// rows k1, the length-N2 DFTs over n2 of the data (R0[n2 N1 + k1]) and of
// the kernel (R1[n2 N1 + k1]) complete both spectra at k = k1 + N1 k2.  The
// inverse transform of their product P starts at once, in LDS: with
// n = n2 + N2 n1 it splits as
//   sum_k P_k W_M^(-n k) = sum_k1 W_N1^(-n1 k1) [W_M^(-n2 k1) sum_k2 W_N2^(-n2 k2) P_(k1 + N1 k2)],
// and the bracket's conjugate, i.e. the forward length-N2 DFT of conj(P)
// times W_M^(+n2 k1) (W_M = e^(-2 pi i / M)), is stored in place at n2 N1 + k1.
template <int E2>
__device__ __forceinline__ void rag_rows_conv(const RagSize &z, int M, CF *smem, float2 *R0, const float2 *R1)
{
    const int N1 = z.N1, RR = z.RR, T2 = z.T2;
    const int tid = (int)threadIdx.x;
    const int r = tid % RR, t = tid / RR;
    CF *lds = smem + (size_t)r * lds_elems(z.N2);
    for (int k10 = 0; k10 < N1; k10 += RR) {
        const int k1 = k10 + r;
        const bool rowok = k1 < N1;
        CF v[E2], w[E2];
#pragma unroll
        for (int e = 0; e < E2; ++e) {
            const size_t i = (size_t)(t + T2 * e) * N1 + k1;
            v[e] = rowok ? ldc<float>(R0 + i) : CF{0.f, 0.f};
            w[e] = rowok ? ldc<float>(R1 + i) : CF{0.f, 0.f};
        }
        fft_lds<E2>(v, lds, t, T2, z.sc2);
        fft_lds<E2>(w, lds, t, T2, z.sc2);
#pragma unroll
        for (int e = 0; e < E2; ++e)
            v[e] = cconj(cmul(v[e], w[e]));
        fft_lds<E2>(v, lds, t, T2, z.sc2);
        // position n2 = t + T2 e: the inverse's twiddle W_M^(-n2 k1), applied to
        // the conjugate as W_M^(+n2 k1) = e^(-2 pi i n2 k1 / M)
        const double A = -(double)umod24(k1 * t, M) / (double)M;
        const double B = -(double)umod24(k1 * T2, M) / (double)M;
        if (rowok) {
#pragma unroll
            for (int e = 0; e < E2; ++e)
                stc<float>(R0 + (size_t)(t + T2 * e) * N1 + k1,
                           cmul(v[e], cis_turns_from<float>(frac_turns(fma(B, (double)e, A)))));
        }
    }
    __syncthreads();
}

// Closing column pass of the inverse transform: for every tile of C
// columns n2, the length-N1 DFT over k1 of the contiguous src[n2 N1 + k1];
// the result at n1 belongs to output index j = n2 + N2 n1 and is handed,
// transposed through LDS so that consecutive threads own consecutive j, to
// `store(j, value)`.
template <int E1, class Store>
__device__ __forceinline__ void rag_icols(const RagSize &z, CF *smem, const float2 *src, Store store)
{
    const int N1 = z.N1, N2 = z.N2, Cc = z.C, T1 = z.T1;
    const int tid = (int)threadIdx.x;
    const int sl = tid / T1, t = tid - sl * T1;
    const int sl2 = tid % Cc, t2 = tid / Cc;
    CF *lds = smem + (size_t)sl * lds_elems(N1);
    const CF *l2 = smem + (size_t)sl2 * lds_elems(N1);
    for (int n20 = 0; n20 < N2; n20 += Cc) {
        const int n2 = n20 + sl;
        const bool colok = n2 < N2;
        CF v[E1];
#pragma unroll
        for (int e = 0; e < E1; ++e)
            v[e] = colok ? ldc<float>(src + (size_t)n2 * N1 + t + T1 * e) : CF{0.f, 0.f};
        fft_lds<E1>(v, lds, t, T1, z.sc1);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E1; ++e)
            lds[lds_pad(t + T1 * e)] = v[e];
        __syncthreads();
        if (n20 + sl2 < N2) {
            store.begin(n20 + sl2 + N2 * t2, N2 * T1);
#pragma unroll
            for (int e = 0; e < E1; ++e)
                store(n20 + sl2 + N2 * (t2 + T1 * e), l2[lds_pad(t2 + T1 * e)], e);
        }
    }
    __syncthreads();
}

// Functors of the column / row passes.
struct PreChirpLoad { // pre-chirped input samples
    const float2 *src;
    LctConst k;
    int N, N2, T1;
    double inv2N;
    ThreadChirp c;
    __device__ void begin(int t, int n2) { c = seq_chirp(k.pre_hi, k.pre_lo, true, t * N2 + n2, T1 * N2, N, inv2N); }
    __device__ CF operator()(int i, int e) const { return cmul(ldc<float>(src + i), chirp_at<float>(c, e)); }
};
struct PostChirpStore { // post-chirped outputs at k2 N1 + k1
    float2 *dst;
    LctConst k;
    int N, N1, T2;
    double inv2N;
    float mag;
    ThreadChirp c;
    __device__ void begin(int k1, int t)
    {
        c = seq_chirp(k.post_hi, k.post_lo, true, k1 + N1 * t, N1 * T2, N, inv2N, k.amp_turns);
    }
    __device__ void operator()(int k1, int k2, CF y, int e) const
    {
        stc<float>(dst + (size_t)k2 * N1 + k1, cscale(cmul(y, chirp_at<float>(c, e)), mag));
    }
};
struct GaussData { // e^{-P x_i^2} f_i (reversed for the Hankel form), zero beyond N
    const float2 *src;
    FrConst k;
    int N, N2, T1;
    GaussPoly g;
    // positions i = (t + T1 e) N2 + n2: n_i = 2i - N + 1 is linear in e
    __device__ void begin(int t, int n2) { g = gauss_poly(k.dmag, k.dph_hi, k.dph_lo, 2 * (t * N2 + n2) - N + 1, 2 * T1 * N2); }
    __device__ CF operator()(int i, int e) const
    {
        CF x = {0.f, 0.f};
        if (i < N)
            x = cmul(ldc<float>(src + (k.hankel ? N - 1 - i : i)), gauss_at(g, e));
        return x;
    }
};
struct GaussKernel { // Toeplitz kernel at circular position i
    double kmag, kph_hi, kph_lo;
    int N, L, N2, T1;
    GaussPoly lo, hi;
    // m = i up to N, L - i beyond; i = (t N2 + n2) + T1 N2 e
    __device__ void begin(int t, int n2)
    {
        lo = gauss_poly(kmag, kph_hi, kph_lo, t * N2 + n2, T1 * N2);
        hi = gauss_poly(kmag, kph_hi, kph_lo, L - (t * N2 + n2), -T1 * N2);
    }
    __device__ CF operator()(int i, int e) const { return i <= N ? gauss_at(lo, e) : gauss_at(hi, e); }
};
struct FrOutStore { // the first N outputs: conjugate, diagonal e^{-P x_j^2}, constant
    float2 *dst;
    double dmag, dph_hi, dph_lo, cre, cim;
    int N;
    GaussPoly g;
    // outputs j = j0 + D e: n_j = 2j - N + 1 linear in e
    __device__ void begin(int j0, int D) { g = gauss_poly(dmag, dph_hi, dph_lo, 2 * j0 - N + 1, 2 * D); }
    __device__ void operator()(int j, CF y, int e) const
    {
        if (j < N) {
            CF o = cmul(cconj(y), gauss_at(g, e));
            stc<float>(dst + j, cmul(o, CF{(float)cre, (float)cim}));
        }
    }
};

template <int E1, int E2>
__device__ __noinline__ void rag_lct_big(const RagArgs &a, const RagItem &it, const RagSize &z, CF *smem)
{
    const int s = a.sig[it.first];
    const RagDesc d = a.desc[s];
    const int N = z.N;
    const float2 *src = a.in + d.offset;
    float2 *dst = a.out + d.offset;
    const double inv2N = 0.5 / (double)N;
    const LctConst k = lct_const_from(z.nc, d.p[0], d.p[1], d.p[2], d.p[3]);
    const float mag = (float)k.amp_mag;
    if (k.b0) {
        const int i0 = (int)threadIdx.x;
        const ThreadChirp cb = thread_chirp(k.post_hi, k.post_lo, false, i0, RAG_THREADS, N, inv2N, k.amp_turns);
        for (int e = 0; i0 + RAG_THREADS * e < N; ++e)
            stc<float>(dst + i0 + RAG_THREADS * e,
                       cmul(ldc<float>(src + i0 + RAG_THREADS * e), cscale(chirp_at<float>(cb, e), mag)));
        __syncthreads();
        return;
    }
    rag_cols<E1>(z, N, smem, dst, PreChirpLoad{src, k, N, z.N2, z.T1, inv2N, {}});
    rag_rows<E2>(z, smem, dst, PostChirpStore{dst, k, N, z.N1, z.T2, inv2N, mag, {}});
}

template <int E1, int E2>
__device__ __noinline__ void rag_frft_big(const RagArgs &a, const RagItem &it, const RagSize &z, CF *smem)
{
    const int s = a.sig[it.first];
    const RagDesc d = a.desc[s];
    const int N = z.N, L = 2 * N;
    const float2 *src = a.in + d.offset;
    float2 *dst = a.out + d.offset;
    float2 *R0 = a.ws + a.wsoff[s];
    float2 *R1 = R0 + L;
    const FrConst k = fr_const(N, d.p[0], d.p[1], false);
    if (k.special) {
        for (int j = (int)threadIdx.x; j < N; j += RAG_THREADS)
            stc<float>(dst + j, cscale(ldc<float>(src + (k.special == 1 ? j : N - 1 - j)), (float)k.cre));
        __syncthreads();
        return;
    }
    rag_cols<E1>(z, L, smem, R0, GaussData{src, k, N, z.N2, z.T1, {}});
    rag_cols<E1>(z, L, smem, R1, GaussKernel{k.kmag, k.kph_hi, k.kph_lo, N, L, z.N2, z.T1, {}, {}});
    rag_rows_conv<E2>(z, L, smem, R0, R1);
    rag_icols<E1>(z, smem, R0, FrOutStore{dst, k.dmag, k.dph_hi, k.dph_lo, k.cre, k.cim, N, {}});
}

#define RAG_E_LIST(X) X(16) X(20) X(24)

template <int E1>
__device__ void rag_big_dispatch(int kind, int E2, const RagArgs &a, const RagItem &it, const RagSize &z, CF *smem)
{
    switch (E2) {
#define X(e2)                                                                                                        \
    case e2:                                                                                                         \
        if (kind == RI_LCT_BIG)                                                                                      \
            rag_lct_big<E1, e2>(a, it, z, smem);                                                                     \
        else                                                                                                         \
            rag_frft_big<E1, e2>(a, it, z, smem);                                                                    \
        break;
        RAG_E_LIST(X)
#undef X
    default:
        break;
    }
}

__global__ __launch_bounds__(RAG_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void k_ragged(RagArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CF *smem = reinterpret_cast<CF *>(smem_raw);
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0)
            next = atomicAdd(a.head, 1);
        __syncthreads();
        const int i = next;
        __syncthreads(); // everyone has read `next` before it is overwritten
        if (i >= a.nitems)
            break;
        const RagItem it = a.items[i];
        const RagSize &z = a.sizes[it.size];
        if (it.kind == RI_LCT_GROUP || it.kind == RI_FRFT_GROUP) {
            switch (z.E) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        if (it.kind == RI_LCT_GROUP)                                                                                 \
            rag_lct_group<e>(a, it, z, smem);                                                                        \
        else                                                                                                         \
            rag_frft_group<e>(a, it, z, smem);                                                                       \
        break;
                RAG_E_LIST(X)
#undef X
            default:
                break;
            }
        } else {
            switch (z.E1) {
#define X(e)                                                                                                         \
    case e:                                                                                                          \
        rag_big_dispatch<e>(it.kind, z.E2, a, it, z, smem);                                                          \
        break;
                RAG_E_LIST(X)
#undef X
            default:
                break;
            }
        }
        __syncthreads(); // LDS is reused by the next item
    }
}

__global__ void k_ragged_reset(int *head)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *head = 0;
}

} // namespace lctk
