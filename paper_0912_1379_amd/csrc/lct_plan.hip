// lct_plan.hip - launch geometry: the built-in heuristic, the candidate
// geometries, and the autotuner that times the candidates on the device and
// records the fastest per (transform kind, length, precision) in a
// process-wide table that the entry points consult.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lct.h"
#include "plan.hpp"

namespace lctk {

bool smooth235(int64_t N)
{
    if (N < 1 || N > MAX_N)
        return false;
    for (int p : {2, 3, 5})
        while (N % p == 0)
            N /= p;
    return N == 1;
}

// Largest 2^p 3^q 5^r length whose padded LDS image fits 160 KiB with at
// most 1024 threads.
int64_t single_pass_limit(bool fp64) { return fp64 ? 8192 : 16384; }

namespace {

const int E_WIDTHS[] = {
#define X(e) e,
    LCT_E_LIST(X)
#undef X
};
const int RADICES[] = {16, 8, 5, 4, 3, 2};

bool e_instantiated(int E)
{
    for (int e : E_WIDTHS)
        if (e == E)
            return true;
    return false;
}

bool sched_valid(const Sched &sc, int64_t Nfft, int E)
{
    if (sc.nst < 0 || sc.nst > 24)
        return false;
    int64_t prod = 1;
    for (int s = 0; s < sc.nst; ++s) {
        bool known = false;
        for (int r : RADICES)
            known |= sc.rad[s] == r;
        if (!known || E % sc.rad[s] != 0)
            return false;
        prod *= sc.rad[s];
        if (prod > Nfft)
            return false;
    }
    return prod == Nfft;
}

// Greedy schedule over the allowed radices (largest first); `rev` runs the
// same stages in the opposite order.
bool same_sched(const Sched &a, const Sched &b)
{
    if (a.nst != b.nst)
        return false;
    for (int s = 0; s < a.nst; ++s)
        if (a.rad[s] != b.rad[s])
            return false;
    return true;
}

// Elements per thread: the first E of the list for the size's prime set that
// divides N and keeps the thread count per signal within a work-group.
int choose_E(int64_t N, bool fp64, bool frft)
{
    int64_t m = N;
    bool p2 = false, p3 = false, p5 = false;
    while (m % 2 == 0) { m /= 2; p2 = true; }
    while (m % 3 == 0) { m /= 3; p3 = true; }
    while (m % 5 == 0) { m /= 5; p5 = true; }
    static const int l2[] = {16, 8, 4, 2, 0};
    static const int l3[] = {27, 9, 3, 0};
    static const int l5[] = {25, 5, 0};
    static const int l23[] = {24, 12, 6, 18, 0};
    static const int l25[] = {20, 10, 0};
    static const int l35[] = {15, 0};
    static const int l235[] = {30, 0};
    static const int l1[] = {1, 0};
    static const int l23_64[] = {12, 6, 24, 18, 0};
    static const int l25_64[] = {10, 20, 0};
    static const int l2_fr64[] = {8, 16, 4, 2, 0}; // FP64 two-pass convolution rows
    const int *lst;
    if (p2 && p3 && p5) lst = l235;
    else if (p2 && p3) lst = fp64 ? l23_64 : l23;
    else if (p2 && p5) lst = fp64 ? l25_64 : l25;
    else if (p3 && p5) lst = l35;
    else if (p2) lst = (frft && fp64) ? l2_fr64 : l2;
    else if (p3) lst = l3;
    else if (p5) lst = l5;
    else lst = l1;
    for (int i = 0; lst[i]; ++i) {
        const int E = lst[i];
        if (N % E == 0 && N / E <= max_block(fp64, E))
            return E;
    }
    return 0;
}

// Columns (or rows) per four-step work-group: as many as keep >= 128-byte
// row segments, about 256 threads, and fit LDS and the launch bound, capped
// at `cap_limit` (smaller groups trade row-segment length for more resident
// work-groups per CU; neighbouring groups then share lines in one L2).
int pick_group(int Nsub, int T, int E, int other, bool fp64, int cap_limit)
{
    const size_t elem = fp64 ? 16 : 8;
    const size_t per = (size_t)lds_elems(Nsub) * elem;
    const int want = fp64 ? 8 : 16;
    int cap = 256 / T > want ? 256 / T : want;
    if (cap > cap_limit)
        cap = cap_limit;
    for (int c = cap; c >= 1; --c) {
        if (other % c)
            continue;
        if (c * T > max_block(fp64, E) || c * per > LDS_BYTES)
            continue;
        return c;
    }
    return 0;
}

} // namespace

Sched greedy_sched(int64_t N, int E, int maxrad, bool rev)
{
    Sched s{};
    int64_t rem = N;
    while (rem > 1 && s.nst < 24) {
        bool ok = false;
        for (int c : {16, 8, 5, 4, 3, 2}) {
            if (c <= maxrad && E % c == 0 && rem % c == 0) {
                s.rad[s.nst++] = c;
                rem /= c;
                ok = true;
                break;
            }
        }
        if (!ok)
            break;
    }
    if (rem != 1) {
        s.nst = -1;
        return s;
    }
    if (rev)
        for (int i = 0, j = s.nst - 1; i < j; ++i, --j) {
            const int x = s.rad[i];
            s.rad[i] = s.rad[j];
            s.rad[j] = x;
        }
    return s;
}



Tiling tiling_of(int64_t Nfft, bool fp64, int E, int S, const Sched &sc, size_t extra)
{
    Tiling t;
    if (Nfft < 1 || Nfft > single_pass_limit(fp64) || !e_instantiated(E) || Nfft % E != 0 || S < 1)
        return t;
    t.E = E;
    t.T = (int)(Nfft / E);
    t.S = S;
    t.sc = sc;
    if (!sched_valid(sc, Nfft, E))
        return t;
    const size_t per = (size_t)lds_elems((int)Nfft) * (fp64 ? 16 : 8) + extra;
    if ((int64_t)S * t.T > max_block(fp64, E) || (size_t)S * per > LDS_BYTES)
        return t;
    t.block = S * t.T;
    t.lds = (size_t)S * per;
    t.ok = true;
    return t;
}

Tiling default_tiling(int64_t Nfft, bool fp64, bool frft, size_t extra)
{
    // The single-pass convolution takes the LCT's widths: in FP64, 16 values
    // per thread on half the threads fit the registers where 8 on 1024
    // threads spilled.  (The two-pass convolution's rows keep FP64 at 8
    // first: choose_E with frft set.)
    (void)frft;
    const int E = choose_E(Nfft, fp64, false);
    if (E == 0)
        return Tiling{};
    const int T = (int)(Nfft / E);
    const size_t per = (size_t)lds_elems((int)Nfft) * (fp64 ? 16 : 8) + extra;
    int S = T >= 256 ? 1 : 256 / T;
    while (S > 1 && (size_t)S * per > LDS_BYTES)
        --S;
    return tiling_of(Nfft, fp64, E, S, greedy_sched(Nfft, E, 16, false), extra);
}

FsTiling fs_of(int64_t N, bool fp64, int N1, int E1, int E2, int C, int RR, const Sched &sc1, const Sched &sc2)
{
    FsTiling f;
    if (N1 < 2 || N % N1 != 0)
        return f;
    const int64_t N2 = N / N1;
    if (N2 < 2 || C < 1 || RR < 1 || N2 % C != 0 || N1 % RR != 0)
        return f;
    const Tiling a = tiling_of(N1, fp64, E1, C, sc1, 0), b = tiling_of(N2, fp64, E2, RR, sc2, 0);
    if (!a.ok || !b.ok)
        return f;
    f.N1 = N1;
    f.N2 = (int)N2;
    f.E1 = E1;
    f.E2 = E2;
    f.T1 = a.T;
    f.T2 = b.T;
    f.C = C;
    f.RR = RR;
    f.bs1 = a.block;
    f.bs2 = b.block;
    f.lds1 = a.lds;
    f.lds2 = b.lds;
    f.sc1 = sc1;
    f.sc2 = sc2;
    f.ok = true;
    return f;
}

namespace {

bool pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

} // namespace

Tiling mfma_tiling(int64_t N)
{
    if (!pow2(N) || N < 256 || N > single_pass_limit(false))
        return Tiling{};
    const int T = (int)(N / 16);
    const int S = T >= 256 ? 1 : 256 / T;
    Tiling t = tiling_of(N, false, 16, S, greedy_sched(N, 16, 16, false), 0);
    t.mf = t.ok && t.block % 64 == 0;
    t.ok = t.mf;
    return t;
}

FsTiling mfma_fs(int64_t N)
{
    if (!pow2(N) || N <= single_pass_limit(false) || N > MAX_N)
        return FsTiling{};
    int lg = 0;
    while ((int64_t(1) << lg) < N)
        ++lg;
    const int64_t N1 = int64_t(1) << (lg / 2), N2 = N / N1;
    // 256-thread work-groups: 256 / (N1 / 16) columns, 256 / (N2 / 16) rows
    // (neighbouring tiles share an L2 through the XCD-aware tile order)
    const int C = (int)std::max<int64_t>(1, 256 / (N1 / 16));
    const int RR = (int)std::max<int64_t>(1, 256 / (N2 / 16));
    FsTiling f = fs_of(N, false, (int)N1, 16, 16, C, RR, greedy_sched(N1, 16, 16, false),
                       greedy_sched(N2, 16, 16, false));
    if (!f.ok)
        return f;
    f.mf1 = N1 % 256 == 0 && f.bs1 % 64 == 0;
    f.mf2 = N2 % 256 == 0 && f.bs2 % 64 == 0;
    return f;
}

namespace {

// max_threads bounds each pass's work-group (columns or rows times threads
// per column or row), except that at least min_group columns or rows are
// allowed.
FsTiling fs_for_split(int64_t N, bool fp64, int64_t N1, int E1, int E2, int cap, int max_threads = 1024,
                      int min_group = 1)
{
    const int64_t N2 = N / N1;
    if (!E1 || !E2)
        return FsTiling{};
    const int T1 = (int)(N1 / E1), T2 = (int)(N2 / E2);
    const int C = pick_group((int)N1, T1, E1, (int)N2, fp64, std::min(cap, std::max(min_group, max_threads / T1)));
    const int RR =
        pick_group((int)N2, T2, E2, (int)N1, fp64, std::min(cap, std::max(min_group, max_threads / T2)));
    if (!C || !RR)
        return FsTiling{};
    return fs_of(N, fp64, (int)N1, E1, E2, C, RR, greedy_sched(N1, E1, 16, false), greedy_sched(N2, E2, 16, false));
}

} // namespace

// N = N1 N2 with N1 the largest divisor <= sqrt(N) whose tiles fit.  The
// work-groups hold about 256 threads but at least four columns (rows), i.e.
// output segments of 32 bytes or more: timed against every candidate at
// 2^14..2^24 this came within 7.5% of the fastest at all lengths but one
// (FP64 2^14: 12.6%, where the geometry did not change), while the 1024-thread
// groups of 16 columns that the tile-width bound alone gives were up to 25%
// slower.  For the fractional transform's convolution (frft)
// the work-groups stay within 256 threads, and pass 2, which holds a row of
// the data's and of the kernel's values per thread, takes a factor whose width
// has the 256-thread instantiation (16 FP32, 8 FP64), the shorter one when
// both factors do.
FsTiling default_fs(int64_t N, bool fp64, bool frft)
{
    int64_t best = 0;
    for (int64_t d = 1; d * d <= N; ++d)
        if (N % d == 0)
            best = d;
    if (frft) {
        const int tight = fp64 ? 8 : 16;
        for (int64_t d = best; d >= 2; --d) {
            if (N % d)
                continue;
            for (const int64_t N2 : {d, N / d}) {
                const int64_t N1 = N / N2;
                if (N1 > single_pass_limit(fp64) || N2 > single_pass_limit(fp64))
                    continue;
                const int E2 = choose_E(N2, fp64, true);
                if (E2 != tight)
                    continue;
                FsTiling f = fs_for_split(N, fp64, N1, choose_E(N1, fp64, false), E2, 64, 256);
                if (f.ok)
                    return f;
            }
        }
    }
    for (int64_t N1 = best; N1 >= 2; --N1) {
        if (N % N1)
            continue;
        const int64_t N2 = N / N1;
        if (N1 > single_pass_limit(fp64) || N2 > single_pass_limit(fp64))
            break;
        FsTiling f = fs_for_split(N, fp64, N1, choose_E(N1, fp64, false), choose_E(N2, fp64, frft), 64, 256,
                                  frft ? 1 : 4);
        if (f.ok)
            return f;
    }
    return FsTiling{};
}

void tiling_candidates(int64_t Nfft, bool fp64, bool frft, Tiling *out, int *n, int cap)
{
    *n = 0;
    auto push = [&](const Tiling &t) {
        if (!t.ok || *n >= cap)
            return;
        for (int i = 0; i < *n; ++i)
            if (out[i].E == t.E && out[i].S == t.S && same_sched(out[i].sc, t.sc))
                return;
        out[(*n)++] = t;
    };
    push(default_tiling(Nfft, fp64, frft, 0));
    for (int E : E_WIDTHS) {
        if (Nfft % E != 0 || Nfft / E > max_block(fp64, E) || (Nfft > 1 && E == 1) || (Nfft >= 64 && E <= 2))
            continue; // (radix-2-only geometries of non-tiny lengths are never competitive)
        const int T = (int)(Nfft / E);
        const int S0 = T >= 256 ? 1 : 256 / T;
        for (int maxrad : {16, 8})
            for (int rev = 0; rev < 2; ++rev) {
                const Sched sc = greedy_sched(Nfft, E, maxrad, rev != 0);
                if (sc.nst < 0)
                    continue;
                for (int mul : {1, 2, 4}) {
                    push(tiling_of(Nfft, fp64, E, S0 * mul, sc, 0));
                    if (mul == 1 && S0 >= 2)
                        push(tiling_of(Nfft, fp64, E, S0 / 2, sc, 0));
                }
            }
    }
}

void fs_candidates(int64_t Nfft, bool fp64, bool frft, FsTiling *out, int *n, int cap)
{
    *n = 0;
    auto push = [&](const FsTiling &f) {
        if (!f.ok || *n >= cap)
            return;
        for (int i = 0; i < *n; ++i)
            if (out[i].N1 == f.N1 && out[i].E1 == f.E1 && out[i].E2 == f.E2 && out[i].C == f.C &&
                out[i].RR == f.RR && same_sched(out[i].sc1, f.sc1) && same_sched(out[i].sc2, f.sc2))
                return;
        out[(*n)++] = f;
    };
    push(default_fs(Nfft, fp64, frft));
    // splits nearest to sqrt(N) in log distance, both factors within one pass
    std::vector<std::pair<double, int64_t>> splits;
    for (int64_t d = 2; d * 2 <= Nfft; ++d)
        if (Nfft % d == 0 && d <= single_pass_limit(fp64) && Nfft / d <= single_pass_limit(fp64))
            splits.push_back({fabs(log((double)d) - 0.5 * log((double)Nfft)), d});
    std::sort(splits.begin(), splits.end());
    int used = 0;
    for (const auto &sp : splits) {
        if (used++ >= 4)
            break;
        const int64_t N1 = sp.second, N2 = Nfft / N1;
        const int e1 = choose_E(N1, fp64, false), e2 = choose_E(N2, fp64, false);
        for (int cap : {64, 32, 16, 8, 4}) {
            push(fs_for_split(Nfft, fp64, N1, e1, e2, cap));
            if (frft)
                push(fs_for_split(Nfft, fp64, N1, e1, e2, cap, 256));
        }
        for (int E1 : E_WIDTHS)
            for (int E2 : E_WIDTHS) {
                if ((E1 != e1 && E1 * 2 != e1) || (E2 != e2 && E2 * 2 != e2))
                    continue; // the heuristic width and the next smaller one
                push(fs_for_split(Nfft, fp64, N1, E1, E2, 64));
            }
    }
}

// ---------------------------------------------------------------------------
// The table of tuned geometries.  An entry is a text line:
//   <kind> N=<n> prec=<fp32|fp64> E=<e> S=<s> rad=<r.r.r>                 (one pass)
//   <kind> N=<n> prec=<..> N1=<n1> E1=<e1> E2=<e2> C=<c> RR=<rr> rad1=<..> rad2=<..>  (two passes)
// kind is "lct" or "frft"; for "frft" the geometry is that of the length-2N
// convolution.  Lines starting with '#' are comments.
namespace {

struct TuneKey {
    int kind;
    int64_t N;
    bool fp64;
    bool operator<(const TuneKey &o) const { return std::tie(kind, N, fp64) < std::tie(o.kind, o.N, o.fp64); }
};
struct TuneEntry {
    bool two_pass = false;
    Tiling t;
    FsTiling f;
};

std::mutex g_mu;
std::map<TuneKey, TuneEntry> g_table;

std::string rad_text(const Sched &sc)
{
    std::string s;
    for (int i = 0; i < sc.nst; ++i) {
        if (i)
            s += ".";
        s += std::to_string(sc.rad[i]);
    }
    return s;
}

std::string entry_text(const TuneKey &k, const TuneEntry &e)
{
    char buf[256];
    const char *kind = k.kind == LCT_TUNE_FRFT ? "frft" : "lct";
    const char *prec = k.fp64 ? "fp64" : "fp32";
    if (!e.two_pass)
        snprintf(buf, sizeof buf, "%s N=%lld prec=%s E=%d S=%d rad=%s", kind, (long long)k.N, prec, e.t.E, e.t.S,
                 rad_text(e.t.sc).c_str());
    else
        snprintf(buf, sizeof buf, "%s N=%lld prec=%s N1=%d E1=%d E2=%d C=%d RR=%d rad1=%s rad2=%s", kind,
                 (long long)k.N, prec, e.f.N1, e.f.E1, e.f.E2, e.f.C, e.f.RR, rad_text(e.f.sc1).c_str(),
                 rad_text(e.f.sc2).c_str());
    return buf;
}

bool parse_rad(const std::string &v, Sched *sc)
{
    *sc = Sched{};
    if (v.empty())
        return true; // no stages (length 1)
    size_t i = 0;
    while (i < v.size()) {
        size_t j = v.find('.', i);
        if (j == std::string::npos)
            j = v.size();
        const std::string tok = v.substr(i, j - i);
        if (tok.empty() || tok.size() > 3 || sc->nst >= 24)
            return false;
        for (char ch : tok)
            if (ch < '0' || ch > '9')
                return false;
        sc->rad[sc->nst++] = atoi(tok.c_str());
        i = j + 1;
    }
    return v.back() != '.';
}

// Parses and validates one entry; every kernel precondition is checked here,
// so that nothing read from a file can produce an invalid launch.
int parse_entry(const char *line, TuneKey *key, TuneEntry *ent)
{
    std::vector<std::pair<std::string, std::string>> kv;
    std::string kind;
    const char *p = line;
    while (*p) {
        while (*p == ' ' || *p == '\t')
            ++p;
        if (!*p || *p == '\n' || *p == '\r')
            break;
        const char *q = p;
        while (*q && *q != ' ' && *q != '\t' && *q != '\n' && *q != '\r')
            ++q;
        const std::string tok(p, q);
        const size_t eq = tok.find('=');
        if (kind.empty() && eq == std::string::npos)
            kind = tok;
        else if (eq == std::string::npos || eq == 0)
            return LCT_ERR_ARG;
        else
            kv.push_back({tok.substr(0, eq), tok.substr(eq + 1)});
        p = q;
    }
    if (kind != "lct" && kind != "frft")
        return LCT_ERR_ARG;
    for (size_t i = 0; i < kv.size(); ++i) // each field at most once
        for (size_t j = 0; j < i; ++j)
            if (kv[i].first == kv[j].first)
                return LCT_ERR_ARG;
    key->kind = kind == "lct" ? LCT_TUNE_LCT : LCT_TUNE_FRFT;
    long long N = 0;
    int E = 0, S = 0, N1 = 0, E1 = 0, E2 = 0, C = 0, RR = 0;
    Sched sc{}, sc1{}, sc2{};
    bool have_prec = false, have_rad = false, have_rad1 = false, have_rad2 = false;
    for (const auto &x : kv) {
        const std::string &k = x.first, &v = x.second;
        auto num = [&](long long *out) {
            if (v.empty() || v.size() > 12)
                return false;
            for (char ch : v)
                if (ch < '0' || ch > '9')
                    return false;
            *out = atoll(v.c_str());
            return true;
        };
        long long t = 0;
        if (k == "prec") {
            if (v != "fp32" && v != "fp64")
                return LCT_ERR_ARG;
            key->fp64 = v == "fp64";
            have_prec = true;
        } else if (k == "rad") {
            if (!(have_rad = parse_rad(v, &sc)))
                return LCT_ERR_ARG;
        } else if (k == "rad1") {
            if (!(have_rad1 = parse_rad(v, &sc1)))
                return LCT_ERR_ARG;
        } else if (k == "rad2") {
            if (!(have_rad2 = parse_rad(v, &sc2)))
                return LCT_ERR_ARG;
        } else if (!num(&t) || t > (1LL << 30)) {
            return LCT_ERR_ARG;
        } else if (k == "N") {
            N = t;
        } else if (k == "E") {
            E = (int)t;
        } else if (k == "S") {
            S = (int)t;
        } else if (k == "N1") {
            N1 = (int)t;
        } else if (k == "E1") {
            E1 = (int)t;
        } else if (k == "E2") {
            E2 = (int)t;
        } else if (k == "C") {
            C = (int)t;
        } else if (k == "RR") {
            RR = (int)t;
        } else {
            return LCT_ERR_ARG;
        }
    }
    if (!have_prec || !smooth235(N))
        return LCT_ERR_ARG;
    key->N = N;
    const int64_t Nfft = key->kind == LCT_TUNE_FRFT ? 2 * N : N;
    const bool two = Nfft > single_pass_limit(key->fp64);
    ent->two_pass = two;
    if (!two) {
        if (!have_rad || have_rad1 || have_rad2)
            return LCT_ERR_ARG;
        ent->t = tiling_of(Nfft, key->fp64, E, S, sc, 0);
        return ent->t.ok ? LCT_OK : LCT_ERR_ARG;
    }
    if (!have_rad1 || !have_rad2 || have_rad)
        return LCT_ERR_ARG;
    ent->f = fs_of(Nfft, key->fp64, N1, E1, E2, C, RR, sc1, sc2);
    return ent->f.ok ? LCT_OK : LCT_ERR_ARG;
}

int load_table(const char *path);

// LCT_TUNE_CACHE: a table file read before the first lookup (again whenever
// the variable names another file).  A missing or invalid file leaves the
// table as it is; lct_tune_clear does not cause a reload.
void cache_load()
{
    const char *path = getenv("LCT_TUNE_CACHE");
    if (!path || !*path)
        return;
    static std::mutex m;
    static std::string loaded;
    std::lock_guard<std::mutex> g(m);
    if (loaded == path)
        return;
    loaded = path;
    (void)load_table(path);
}

// After an autotune: the whole table to LCT_TUNE_CACHE, through a temporary
// file renamed over it so that a reader never sees half a table.
void cache_save()
{
    const char *path = getenv("LCT_TUNE_CACHE");
    if (!path || !*path)
        return;
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    if (lct_tune_save(tmp.c_str()) == LCT_OK && rename(tmp.c_str(), path) != 0)
        (void)remove(tmp.c_str());
}

bool lookup(int kind, int64_t N, bool fp64, TuneEntry *e)
{
    cache_load();
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_table.find(TuneKey{kind, N, fp64});
    if (it == g_table.end())
        return false;
    *e = it->second;
    return true;
}

} // namespace

Tiling select_tiling(int kind, int64_t N, int64_t Nfft, bool fp64, size_t extra)
{
    TuneEntry e;
    if (lookup(kind, N, fp64, &e) && !e.two_pass) {
        Tiling t = tiling_of(Nfft, fp64, e.t.E, e.t.S, e.t.sc, extra);
        if (t.ok)
            return t;
    }
    return default_tiling(Nfft, fp64, kind == LCT_TUNE_FRFT, extra);
}

FsTiling select_fs(int kind, int64_t N, int64_t Nfft, bool fp64)
{
    TuneEntry e;
    if (lookup(kind, N, fp64, &e) && e.two_pass && e.f.ok)
        return e.f;
    return default_fs(Nfft, fp64, kind == LCT_TUNE_FRFT);
}

void autotune_on_plan(int64_t N, int prec)
{
    const char *v = getenv("LCT_AUTOTUNE");
    if (!v || strcmp(v, "1") != 0 || (prec != LCT_FP32 && prec != LCT_FP64))
        return;
    const bool fp64 = prec == LCT_FP64;
    for (int kind : {LCT_TUNE_LCT, LCT_TUNE_FRFT}) {
        TuneEntry e;
        if (!lookup(kind, N, fp64, &e))
            (void)lct_autotune(N, (lct_precision)prec, kind, 0, nullptr, nullptr); // failure keeps the heuristic
    }
}

} // namespace lctk

using namespace lctk;

namespace {

constexpr int MAX_CAND = 96;

struct Bufs {
    void *in = nullptr, *out = nullptr, *par = nullptr, *ws = nullptr;
    ~Bufs()
    {
        (void)hipFree(in);
        (void)hipFree(out);
        (void)hipFree(par);
        (void)hipFree(ws);
    }
};

// Mean time of one launch sequence (all passes) over `reps` runs, in
// microseconds; negative if a launch failed.
template <class F> double time_it(F run, hipStream_t s, int reps)
{
    for (int w = 0; w < 2; ++w)
        if (run() != LCT_OK)
            return -1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return -1.0;
    }
    double us = -1.0;
    bool ok = hipEventRecord(e0, s) == hipSuccess;
    for (int r = 0; ok && r < reps; ++r)
        ok = run() == LCT_OK;
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
        us = 1000.0 * ms / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return us;
}

} // namespace

namespace lctk {
namespace {

// Reads a table file: every non-comment line must be a valid entry (a line
// longer than the buffer is invalid), else nothing is taken from the file.
int load_table(const char *path)
{
    if (!path)
        return LCT_ERR_ARG;
    FILE *f = fopen(path, "r");
    if (!f)
        return LCT_ERR_ARG;
    std::vector<std::pair<TuneKey, TuneEntry>> got;
    char line[512];
    int rc = LCT_OK;
    while (fgets(line, sizeof line, f)) {
        const size_t len = strlen(line);
        if (len == sizeof line - 1 && line[len - 1] != '\n' && !feof(f)) {
            rc = LCT_ERR_ARG;
            break;
        }
        const char *p = line;
        while (*p == ' ' || *p == '\t')
            ++p;
        if (*p == '#' || *p == '\n' || *p == '\r' || *p == 0)
            continue;
        TuneKey k{};
        TuneEntry e;
        if ((rc = parse_entry(p, &k, &e)) != LCT_OK)
            break;
        got.push_back({k, e});
    }
    fclose(f);
    if (rc != LCT_OK)
        return rc;
    std::lock_guard<std::mutex> g(g_mu);
    for (const auto &kv : got)
        g_table[kv.first] = kv.second;
    return LCT_OK;
}

} // namespace
} // namespace lctk

extern "C" {

int lct_tune_candidates(int64_t N, lct_precision prec, int kind, char *buf, size_t cap, int *count)
{
    if ((prec != LCT_FP32 && prec != LCT_FP64) || (kind != LCT_TUNE_LCT && kind != LCT_TUNE_FRFT))
        return LCT_ERR_ARG;
    if (!smooth235(N))
        return LCT_ERR_UNSUPPORTED_N;
    const bool fp64 = prec == LCT_FP64;
    const int64_t Nfft = kind == LCT_TUNE_FRFT ? 2 * N : N;
    const TuneKey key{kind, N, fp64};
    std::string text;
    int n = 0;
    if (Nfft <= single_pass_limit(fp64)) {
        Tiling c[MAX_CAND];
        tiling_candidates(Nfft, fp64, kind == LCT_TUNE_FRFT, c, &n, MAX_CAND);
        for (int i = 0; i < n; ++i) {
            TuneEntry e;
            e.t = c[i];
            text += entry_text(key, e) + "\n";
        }
    } else {
        FsTiling c[MAX_CAND];
        fs_candidates(Nfft, fp64, kind == LCT_TUNE_FRFT, c, &n, MAX_CAND);
        for (int i = 0; i < n; ++i) {
            TuneEntry e;
            e.two_pass = true;
            e.f = c[i];
            text += entry_text(key, e) + "\n";
        }
    }
    if (count)
        *count = n;
    if (buf) {
        if (cap < text.size() + 1)
            return LCT_ERR_ARG;
        memcpy(buf, text.c_str(), text.size() + 1);
    }
    return LCT_OK;
}

int lct_tune_set(const char *line)
{
    if (!line)
        return LCT_ERR_ARG;
    TuneKey k{};
    TuneEntry e;
    const int rc = parse_entry(line, &k, &e);
    if (rc)
        return rc;
    std::lock_guard<std::mutex> g(g_mu);
    g_table[k] = e;
    return LCT_OK;
}

int lct_tune_get(int64_t N, lct_precision prec, int kind, char *buf, size_t cap)
{
    if ((prec != LCT_FP32 && prec != LCT_FP64) || (kind != LCT_TUNE_LCT && kind != LCT_TUNE_FRFT) || !buf)
        return LCT_ERR_ARG;
    if (!smooth235(N))
        return LCT_ERR_UNSUPPORTED_N;
    const bool fp64 = prec == LCT_FP64;
    const TuneKey key{kind, N, fp64};
    TuneEntry e;
    const int64_t Nfft = kind == LCT_TUNE_FRFT ? 2 * N : N;
    if (!lookup(kind, N, fp64, &e)) {
        // the heuristic's choice
        e.two_pass = Nfft > single_pass_limit(fp64);
        if (e.two_pass)
            e.f = default_fs(Nfft, fp64, kind == LCT_TUNE_FRFT);
        else
            e.t = default_tiling(Nfft, fp64, kind == LCT_TUNE_FRFT, 0);
    }
    const std::string s = entry_text(key, e);
    if (cap < s.size() + 1)
        return LCT_ERR_ARG;
    memcpy(buf, s.c_str(), s.size() + 1);
    return LCT_OK;
}

void lct_tune_clear(void)
{
    std::lock_guard<std::mutex> g(g_mu);
    g_table.clear();
}

int lct_tune_save(const char *path)
{
    if (!path)
        return LCT_ERR_ARG;
    std::string text = "# lct autotune table: one geometry per (transform, length, precision)\n";
    {
        std::lock_guard<std::mutex> g(g_mu);
        for (const auto &kv : g_table)
            text += entry_text(kv.first, kv.second) + "\n";
    }
    FILE *f = fopen(path, "w");
    if (!f)
        return LCT_ERR_ARG;
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    return (fclose(f) == 0 && ok) ? LCT_OK : LCT_ERR_ARG;
}

int lct_tune_load(const char *path) { return load_table(path); }

int lct_autotune(int64_t N, lct_precision prec, int kind, int64_t batch, hipStream_t stream, lct_tune_result *res)
{
    if ((prec != LCT_FP32 && prec != LCT_FP64) || (kind != LCT_TUNE_LCT && kind != LCT_TUNE_FRFT) || batch < 0)
        return LCT_ERR_ARG;
    if (!smooth235(N))
        return LCT_ERR_UNSUPPORTED_N;
    const bool fp64 = prec == LCT_FP64;
    const size_t elem = fp64 ? 16 : 8;
    const int64_t Nfft = kind == LCT_TUNE_FRFT ? 2 * N : N;
    const bool two = Nfft > single_pass_limit(fp64);
    if (batch == 0)
        batch = (int64_t(1) << 24) / N > 0 ? (int64_t(1) << 24) / N : 1;
    const size_t bytes = (size_t)batch * (size_t)N * elem;
    Bufs b;
    if (hipMalloc(&b.in, bytes) != hipSuccess || hipMalloc(&b.out, bytes) != hipSuccess ||
        hipMalloc(&b.par, (size_t)batch * 4 * sizeof(double)) != hipSuccess)
        return LCT_ERR_HIP;
    size_t wsb = 0;
    if (kind == LCT_TUNE_FRFT) {
        // two passes: the convolution workspace; one pass: room for the
        // kernel's spectrum (the shared-order mode, timed beside the other)
        wsb = two ? (size_t)batch * 2 * (size_t)Nfft * elem : (size_t)Nfft * elem;
        if (hipMalloc(&b.ws, wsb) != hipSuccess)
            return LCT_ERR_HIP;
    }
    // inputs: 0.5 + 0.5i in every sample; parameters: (a, b, c, d) =
    // (0.5, 1, -0.5, 1) per signal for the LCT, z = 0.6 e^{-1.1 i} for the
    // fractional transform
    std::vector<double> par((size_t)batch * 4);
    for (int64_t s = 0; s < batch; ++s) {
        if (kind == LCT_TUNE_LCT) {
            par[4 * s] = 0.5;
            par[4 * s + 1] = 1.0;
            par[4 * s + 2] = -0.5;
            par[4 * s + 3] = 1.0;
        } else {
            par[2 * s] = 0.6 * cos(-1.1);
            par[2 * s + 1] = 0.6 * sin(-1.1);
        }
    }
    // every 32-bit word set: 0.5f, or for FP64 the double 0x3fe000003fe00000 (about 0.5)
    const uint32_t pattern = fp64 ? 0x3fe00000u : 0x3f000000u;
    if (hipMemsetD32Async((hipDeviceptr_t)b.in, pattern, bytes / 4, stream) != hipSuccess ||
        hipMemcpyAsync(b.par, par.data(), par.size() * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return LCT_ERR_HIP;
    const double *P = (const double *)b.par;
    const int reps = 10;
    int ncand = 0, best = -1;
    double best_us = 0.0, def_us = -1.0;
    TuneEntry win;
    const TuneKey key{kind, N, fp64};
    if (!two) {
        Tiling c[MAX_CAND];
        tiling_candidates(Nfft, fp64, kind == LCT_TUNE_FRFT, c, &ncand, MAX_CAND);
        // one geometry serves both modes of the single-pass fractional
        // transform (an order per signal; one order with its spectrum computed
        // once), so its candidates are ranked by the sum of the two times
        const FrConst shared = fr_const(N, 0.6 * cos(-1.1), 0.6 * sin(-1.1));
        for (int i = 0; i < ncand; ++i) {
            const Tiling &t = c[i];
            double us = time_it(
                [&]() {
                    return kind == LCT_TUNE_LCT ? lct_launch(t, N, fp64, P, nullptr, 0, b.in, b.out, batch, stream)
                                                : frft_sp_launch(t, N, fp64, P, nullptr, b.in, b.out, batch, stream);
                },
                stream, reps);
            if (kind == LCT_TUNE_FRFT && us > 0) {
                const double us1 = time_it(
                    [&]() { return frft_sp_launch(t, N, fp64, nullptr, &shared, b.in, b.out, batch, stream, b.ws); },
                    stream, reps);
                us = us1 > 0 ? us + us1 : -1.0;
            }
            if (i == 0)
                def_us = us; // the first candidate is the heuristic's
            if (us > 0 && (best < 0 || us < best_us)) {
                best = i;
                best_us = us;
                win.two_pass = false;
                win.t = t;
            }
        }
    } else {
        FsTiling c[MAX_CAND];
        fs_candidates(Nfft, fp64, kind == LCT_TUNE_FRFT, c, &ncand, MAX_CAND);
        for (int i = 0; i < ncand; ++i) {
            const FsTiling &f = c[i];
            const double us = time_it(
                [&]() {
                    return kind == LCT_TUNE_LCT
                               ? fs_launch(f, N, fp64, P, nullptr, 0, b.in, b.out, batch, stream)
                               : frft_large_launch(f, N, fp64, P, nullptr, b.in, b.out, batch, b.ws, stream);
                },
                stream, reps);
            if (i == 0)
                def_us = us;
            if (us > 0 && (best < 0 || us < best_us)) {
                best = i;
                best_us = us;
                win.two_pass = true;
                win.f = f;
            }
        }
    }
    if (hipStreamSynchronize(stream) != hipSuccess)
        return LCT_ERR_HIP;
    if (best < 0)
        return ncand ? LCT_ERR_HIP : LCT_ERR_UNSUPPORTED;
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_table[key] = win;
    }
    cache_save();
    if (res) {
        res->kind = kind;
        res->candidates = ncand;
        res->best_us = best_us;
        res->default_us = def_us;
        res->batch = batch;
        const std::string s = entry_text(key, win);
        snprintf(res->config, sizeof res->config, "%s", s.c_str());
    }
    return LCT_OK;
}

} // extern "C"
