// lct_ragged.hip - the ragged-batch entry points: host-side grouping and LPT
// ordering of the work items, plan-owned device tables, and one persistent
// launch (recorded once per pointer set into a HIP graph).
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/lct.h"
#include "ragged_impl.hpp"

using namespace lctk;

static_assert(sizeof(RagDesc) == sizeof(lct_desc), "descriptor layouts must agree");

struct lct_ragged_s {
    int64_t nsig = 0;
    int nitems = 0;
    size_t lds = 0;
    int grid = 0;
    size_t ws_bytes = 0;
    // plan-owned device tables
    RagItem *d_items = nullptr;
    RagSize *d_sizes = nullptr;
    int *d_sig = nullptr;
    int64_t *d_wsoff = nullptr;
    // recorded launch
    std::mutex mu;
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void *g_desc = nullptr, *g_in = nullptr, *g_out = nullptr, *g_ws = nullptr;
};

namespace {

constexpr size_t RAG_LDS_LIMIT = 64 * 1024;

bool smooth235r(int64_t N)
{
    if (N < 1)
        return false;
    for (int p : {2, 3, 5})
        while (N % p == 0)
            N /= p;
    return N == 1;
}

// Values per thread for a length-n DFT inside a 256-thread work-group:
// 16 for 2^k, 24 for 3 2^k, 20 for 5 2^k (the per-signal thread count n/E
// is then a power of two <= 256); 0 if n is not of that form.
int rag_E(int64_t n)
{
    int64_t m = n;
    while (m % 2 == 0)
        m /= 2;
    int E = m == 1 ? 16 : (m == 3 ? 24 : (m == 5 ? 20 : 0));
    if (!E || n < E || n % E || n / E > RAG_THREADS)
        return 0;
    return E;
}

Sched rag_sched(int64_t n, int E)
{
    Sched s{};
    int64_t rem = n;
    const int cand[6] = {16, 8, 5, 4, 3, 2};
    while (rem > 1 && s.nst < 24) {
        bool ok = false;
        for (int c : cand)
            if (E % c == 0 && rem % c == 0) {
                s.rad[s.nst++] = c;
                rem /= c;
                ok = true;
                break;
            }
        if (!ok)
            break;
    }
    if (rem != 1)
        s.nst = -1;
    return s;
}

// single-pass group for a DFT of length n: slots S = 256 / (n / E)
bool rag_group(int64_t n, RagSize &z)
{
    z.E = rag_E(n);
    if (!z.E)
        return false;
    z.T = (int)(n / z.E);
    z.S = RAG_THREADS / z.T;
    z.sc = rag_sched(n, z.E);
    return z.sc.nst >= 0 && (size_t)z.S * lds_elems((int)n) * 8 <= RAG_LDS_LIMIT;
}

// four-step split of a length-M DFT inside one work-group: M = N1 N2, column
// tiles of C = 256 / T1 and row tiles of RR = 256 / T2 (a partial last tile
// is masked); among the valid splits the one with the least masked work wins
bool rag_split(int64_t M, RagSize &z)
{
    double best = 1e300;
    bool found = false;
    for (int64_t a = 16; a <= M / 16; ++a) {
        if (M % a)
            continue;
        const int64_t b = M / a;
        const int E1 = rag_E(a), E2 = rag_E(b);
        if (!E1 || !E2)
            continue;
        const int T1 = (int)(a / E1), T2 = (int)(b / E2);
        const int Cc = RAG_THREADS / T1, RR = RAG_THREADS / T2;
        if ((size_t)Cc * lds_elems((int)a) * 8 > RAG_LDS_LIMIT || (size_t)RR * lds_elems((int)b) * 8 > RAG_LDS_LIMIT)
            continue;
        const Sched s1 = rag_sched(a, E1), s2 = rag_sched(b, E2);
        if (s1.nst < 0 || s2.nst < 0)
            continue;
        const double waste = (double)((b + Cc - 1) / Cc * Cc) / b + (double)((a + RR - 1) / RR * RR) / a;
        const double balance = fabs(log((double)a / (double)b)) * 1e-3; // prefer a ~ b on ties
        if (waste + balance < best) {
            best = waste + balance;
            found = true;
            z.N1 = (int)a;
            z.N2 = (int)b;
            z.E1 = E1;
            z.E2 = E2;
            z.T1 = T1;
            z.T2 = T2;
            z.C = Cc;
            z.RR = RR;
            z.sc1 = s1;
            z.sc2 = s2;
        }
    }
    return found;
}

size_t item_lds(const RagSize &z, int kind)
{
    if (kind == RI_LCT_GROUP)
        return (size_t)z.S * lds_elems(z.N) * 8;
    if (kind == RI_FRFT_GROUP)
        return (size_t)z.S * lds_elems(2 * z.N) * 8;
    size_t a = (size_t)z.C * lds_elems(z.N1) * 8, b = (size_t)z.RR * lds_elems(z.N2) * 8;
    return a > b ? a : b;
}

double item_cost(const RagSize &z, int kind, int count)
{
    const double n = (double)z.N;
    switch (kind) {
    case RI_LCT_GROUP:
        return count * n * log2(n);
    case RI_FRFT_GROUP:
        return count * 3.0 * 2 * n * log2(2 * n);
    case RI_LCT_BIG:
        return 2.0 * n * log2(n) + 2.0 * n * 8;
    default:
        return 3.0 * 2 * 2 * n * log2(2 * n) + 6.0 * 2 * n * 8;
    }
}

// Validates the host descriptors and classifies every signal: its size class
// (one per (kind, N)), its item kind (a single-pass group or a four-step item)
// and, for long fractional transforms, its offset (complex samples) in the
// workspace after the counter.  Shared by the plan and lct_workspace_size.
int classify(const lct_desc *h_desc, int64_t nsig, int prec, std::vector<RagSize> &sizes, std::vector<int> &size_of,
             std::vector<int> &kind_of, std::vector<int64_t> &wsoff, int64_t &ws_elems)
{
    struct Key {
        int kind;
        int N;
    };
    std::vector<Key> keys;
    ws_elems = 0;
    for (int64_t s = 0; s < nsig; ++s) {
        const lct_desc &d = h_desc[s];
        if (d.prec != prec || d.pad != 0)
            return LCT_ERR_ARG;
        if (d.offset < 0 || !smooth235r(d.N) || d.N > (1 << 24))
            return LCT_ERR_UNSUPPORTED_N;
        if (d.kind == LCT_KIND_LCT) {
            if (!lct_row_finite(d.p[0], d.p[1], d.p[2], d.p[3]))
                return LCT_ERR_ARG;
            if (!lct_row_unimodular(d.p[0], d.p[1], d.p[2], d.p[3]))
                return LCT_ERR_NOT_UNIMODULAR;
        } else if (d.kind == LCT_KIND_FRFT) {
            if (!frft_row_finite(d.p[0], d.p[1]))
                return LCT_ERR_ARG;
            if (!frft_row_in_disc(d.p[0], d.p[1]))
                return LCT_ERR_DOMAIN;
        } else {
            return LCT_ERR_ARG;
        }
        int idx = -1;
        for (size_t q = 0; q < keys.size(); ++q)
            if (keys[q].kind == d.kind && keys[q].N == d.N)
                idx = (int)q;
        if (idx < 0) {
            RagSize z{};
            z.N = d.N;
            z.nc = n_const_host(d.N);
            const int64_t L = d.kind == LCT_KIND_LCT ? d.N : 2 * (int64_t)d.N;
            if (!rag_group(L, z)) {
                z.E = z.T = z.S = 0; // not a single-pass group: two-pass item
                if (!rag_split(L, z))
                    return LCT_ERR_UNSUPPORTED;
            }
            sizes.push_back(z);
            keys.push_back({d.kind, d.N});
            idx = (int)sizes.size() - 1;
        }
        size_of[s] = idx;
        const RagSize &z = sizes[idx];
        const bool group = z.E != 0;
        kind_of[s] = d.kind == LCT_KIND_LCT ? (group ? RI_LCT_GROUP : RI_LCT_BIG)
                                            : (group ? RI_FRFT_GROUP : RI_FRFT_BIG);
        if (kind_of[s] == RI_FRFT_BIG) {
            wsoff[s] = ws_elems;
            ws_elems += 2 * 2 * (int64_t)d.N;
        }
    }
    return LCT_OK;
}

// Workspace bytes: the 256-byte counter block, then 2 x 2N complex64 samples
// per long fractional transform.
size_t ws_bytes_of(int64_t ws_elems) { return 256 + (size_t)ws_elems * 8; }

template <typename T> int upload(T **dst, const std::vector<T> &v)
{
    *dst = nullptr;
    if (v.empty())
        return LCT_OK;
    if (hipMalloc((void **)dst, sizeof(T) * v.size()) != hipSuccess)
        return LCT_ERR_HIP;
    if (hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
        return LCT_ERR_HIP;
    return LCT_OK;
}

void release(lct_ragged_plan p)
{
    if (!p)
        return;
    if (p->gexec)
        (void)hipGraphExecDestroy(p->gexec);
    if (p->cap)
        (void)hipStreamDestroy(p->cap);
    (void)hipFree(p->d_items);
    (void)hipFree(p->d_sizes);
    (void)hipFree(p->d_sig);
    (void)hipFree(p->d_wsoff);
    delete p;
}

} // namespace

extern "C" {

int lct_ragged_plan_create(lct_ragged_plan *out, const lct_desc *h_desc, int64_t nsig, lct_precision prec)
{
    if (out == nullptr)
        return LCT_ERR_ARG;
    *out = nullptr;
    if (nsig < 0 || nsig > INT32_MAX || (nsig > 0 && h_desc == nullptr))
        return LCT_ERR_ARG;
    if (prec != LCT_FP32)
        return (prec == LCT_FP64 || prec == LCT_FP32_SPLITBF16) ? LCT_ERR_UNSUPPORTED : LCT_ERR_ARG;

    std::vector<RagSize> sizes;
    std::vector<int> size_of(nsig), kind_of(nsig);
    std::vector<int64_t> wsoff(nsig, 0);
    int64_t ws_elems = 0;
    if (int rc = classify(h_desc, nsig, prec, sizes, size_of, kind_of, wsoff, ws_elems))
        return rc;

    // items: groups of up to S signals of one (kind, N) in descriptor order,
    // one item per two-pass signal; then LPT order
    std::vector<int> sig;
    std::vector<RagItem> items;
    std::vector<double> cost;
    std::vector<std::vector<int>> members(sizes.size());
    for (int64_t s = 0; s < nsig; ++s)
        members[size_of[s]].push_back((int)s);
    for (size_t zi = 0; zi < sizes.size(); ++zi) {
        const RagSize &z = sizes[zi];
        const std::vector<int> &m = members[zi];
        if (m.empty())
            continue;
        const int kind = kind_of[m[0]];
        const int per = (kind == RI_LCT_GROUP || kind == RI_FRFT_GROUP) ? z.S : 1;
        for (size_t i = 0; i < m.size(); i += per) {
            RagItem it{};
            it.kind = kind;
            it.size = (int)zi;
            it.first = (int)sig.size();
            it.count = (int)std::min<size_t>(per, m.size() - i);
            for (int q = 0; q < it.count; ++q)
                sig.push_back(m[i + q]);
            items.push_back(it);
            cost.push_back(item_cost(z, kind, it.count));
        }
    }
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i)
        order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<RagItem> sorted(items.size());
    size_t lds = 0;
    for (size_t i = 0; i < order.size(); ++i) {
        sorted[i] = items[order[i]];
        lds = std::max(lds, item_lds(sizes[sorted[i].size], sorted[i].kind));
    }

    lct_ragged_plan p = new (std::nothrow) lct_ragged_s;
    if (!p)
        return LCT_ERR_ARG;
    p->nsig = nsig;
    p->nitems = (int)sorted.size();
    p->lds = lds;
    p->ws_bytes = ws_bytes_of(ws_elems);
    int rc;
    if ((rc = upload(&p->d_items, sorted)) || (rc = upload(&p->d_sizes, sizes)) || (rc = upload(&p->d_sig, sig)) ||
        (rc = upload(&p->d_wsoff, wsoff))) {
        release(p);
        return rc;
    }
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        release(p);
        return LCT_ERR_HIP;
    }
    if (lds > 0 && hipFuncSetAttribute((const void *)k_ragged, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
        release(p);
        return LCT_ERR_HIP;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_ragged, RAG_THREADS, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    p->grid = std::max(1, std::min(p->nitems, cus * per_cu));
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
        release(p);
        return LCT_ERR_HIP;
    }
    *out = p;
    return LCT_OK;
}

size_t lct_ragged_workspace_size(lct_ragged_plan p) { return p ? p->ws_bytes : 0; }

int lct_workspace_size(const lct_desc *h_desc, int64_t nsig, size_t *bytes)
{
    if (bytes == nullptr)
        return LCT_ERR_ARG;
    *bytes = 0;
    if (nsig < 0 || nsig > INT32_MAX || (nsig > 0 && h_desc == nullptr))
        return LCT_ERR_ARG;
    const int prec = nsig > 0 ? h_desc[0].prec : LCT_FP32;
    if (prec != LCT_FP32)
        return (prec == LCT_FP64 || prec == LCT_FP32_SPLITBF16) ? LCT_ERR_UNSUPPORTED : LCT_ERR_ARG;
    std::vector<RagSize> sizes;
    std::vector<int> size_of(nsig), kind_of(nsig);
    std::vector<int64_t> wsoff(nsig, 0);
    int64_t ws_elems = 0;
    if (int rc = classify(h_desc, nsig, prec, sizes, size_of, kind_of, wsoff, ws_elems))
        return rc;
    *bytes = ws_bytes_of(ws_elems);
    return LCT_OK;
}

int lct_ragged_info(lct_ragged_plan p, int *nitems, int *grid, size_t *lds_bytes)
{
    if (!p)
        return LCT_ERR_ARG;
    if (nitems)
        *nitems = p->nitems;
    if (grid)
        *grid = p->grid;
    if (lds_bytes)
        *lds_bytes = p->lds;
    return LCT_OK;
}

int lct_exec_ragged(lct_ragged_plan p, const lct_desc *d_desc, const void *in, void *out, void *ws, size_t ws_bytes,
                    hipStream_t stream)
{
    if (!p)
        return LCT_ERR_ARG;
    if (p->nsig == 0 || p->nitems == 0)
        return LCT_OK;
    if (d_desc == nullptr || in == nullptr || out == nullptr || ((uintptr_t)in) % 8 || ((uintptr_t)out) % 8 ||
        ((uintptr_t)d_desc) % 8)
        return LCT_ERR_ARG;
    if (in == out)
        return LCT_ERR_ARG; // two-pass items use `out` as their intermediate
    if (ws == nullptr || ws_bytes < p->ws_bytes || ((uintptr_t)ws) % 256)
        return LCT_ERR_WORKSPACE;
    std::lock_guard<std::mutex> g(p->mu);
    if (!(p->gexec && p->g_desc == d_desc && p->g_in == in && p->g_out == out && p->g_ws == ws)) {
        if (p->gexec) {
            (void)hipGraphExecDestroy(p->gexec);
            p->gexec = nullptr;
        }
        RagArgs a{};
        a.desc = reinterpret_cast<const RagDesc *>(d_desc);
        a.sig = p->d_sig;
        a.items = p->d_items;
        a.sizes = p->d_sizes;
        a.wsoff = p->d_wsoff;
        a.nitems = p->nitems;
        a.head = reinterpret_cast<int *>(ws);
        a.in = reinterpret_cast<const float2 *>(in);
        a.out = reinterpret_cast<float2 *>(out);
        a.ws = reinterpret_cast<float2 *>(reinterpret_cast<char *>(ws) + 256);
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return LCT_ERR_HIP;
        hipLaunchKernelGGL(k_ragged_reset, dim3(1), dim3(64), 0, p->cap, a.head);
        hipLaunchKernelGGL(k_ragged, dim3(p->grid), dim3(RAG_THREADS), p->lds, p->cap, a);
        hipError_t le = hipGetLastError();
        hipError_t ce = hipStreamEndCapture(p->cap, &graph);
        if (le != hipSuccess || ce != hipSuccess || graph == nullptr) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return LCT_ERR_HIP;
        }
        hipError_t ie = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            p->gexec = nullptr;
            return LCT_ERR_HIP;
        }
        p->g_desc = d_desc;
        p->g_in = in;
        p->g_out = out;
        p->g_ws = ws;
    }
    return hipGraphLaunch(p->gexec, stream) == hipSuccess ? LCT_OK : LCT_ERR_HIP;
}

void lct_ragged_plan_destroy(lct_ragged_plan p) { release(p); }

} // extern "C"
