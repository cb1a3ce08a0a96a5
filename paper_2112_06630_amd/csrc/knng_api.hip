// Host orchestrator and C ABI (include/knng.h) of the gfx950 NN-Descent library.
//
// One build: pad rows -> random initial graph (Sec. 2) -> iterations of
// {reverse bucketing + weighted sampling (Sec. 3.1), local join (Sec. 2,
// Sec. 3.3), top-K merge} until changes < delta*N*K (Sec. 2) -> optional
// graph-ordered permutation after iteration 1 (Sec. 3.2) -> write-out in
// original order. All device memory comes from the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <utility>
#include <vector>
#include <cstring>
#include <mutex>
#include <array>
#include <cstddef>
#include <string>

#include "knng.h"
#include "knng_impl.h"

using namespace knng;

namespace {

thread_local std::string g_err;

knng_status fail(knng_status s, const std::string& m) {
    g_err = m;
    return s;
}

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
uint64_t host_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Stream state of H(seed, tag, t, ., .): the device finishes the hash with
// one more mix64 of (state ^ (a << 32 | b)).
uint64_t stream_state(uint64_t seed, uint64_t tag, uint64_t t) {
    return host_mix64(host_mix64(seed + 0x9E3779B97F4A7C15ull * (tag + 1)) ^ t);
}

int32_t sample_cap(int32_t K, double rho) {
    const double r = std::ceil(rho * (double)K);
    int32_t c = (int32_t)r;
    if (c < 1) c = 1;
    if (c > K) c = K;
    return c;
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct Plan {
    int path;        // resolved knng_path
    int reorder;
    int bf16;        // BF16-screened precision form
    int dp;
    int split;       // split-BF16 copies of the rows
    int turbo;       // turbosampling coin (knng_sampling)
    int rev_shift, rev_S, rev_B, rev_E;   // counting-sort reverse bucketing (rev_S = 0: atomics)
    int C;
    int64_t pmax;    // proposal slots
    size_t total;
    // byte offsets
    size_t o_Xp, o_nrm, o_nrm64, o_nrm64_2, o_orig, o_posof, o_lkey, o_lpos, o_kth, o_kth2, o_cnt4, o_roff, o_rev, o_cand, o_nn, o_big, o_hubs, o_poff,
        o_pkey, o_scan, o_counters, o_partial, o_Xb, o_nb, o_Xb2, o_nb2, o_comp, o_comp2, o_par, o_lvl, o_best, o_size, o_offs,
        o_cur, o_newpos, o_lkey2, o_lpos2, o_Xp2, o_nrm2, o_orig2, o_flag, o_Xs, o_Xs2, o_rev_h, o_rev_hs, o_rev_tmp,
        o_rk, o_rk2, o_pdone;
    int rowkey = 0;  // RowKey records (low-d direct form of a single build)
};

knng_status validate(int64_t N, int32_t d, const knng_params* p) {
    if (!p) return fail(KNNG_EINVAL, "params is NULL");
    if (N < 2 || N > 0x7ffffffeLL) return fail(KNNG_EINVAL, "N must be in [2, 2^31 - 2]");
    if (d < 1) return fail(KNNG_EINVAL, "d must be >= 1");
    if (p->K < 1 || p->K > 64) return fail(KNNG_EINVAL, "K must be in [1, 64]");
    if ((int64_t)p->K > N - 1) return fail(KNNG_EINVAL, "K must be <= N - 1");
    if (!(p->rho > 0.0) || p->rho > 1.0) return fail(KNNG_EINVAL, "rho must be in (0, 1]");
    if (!(p->delta >= 0.0) || !std::isfinite(p->delta)) return fail(KNNG_EINVAL, "delta must be finite and >= 0");
    if (p->max_iters < 0 || p->max_iters > KNNG_MAX_ITERS)
        return fail(KNNG_EINVAL, "max_iters must be in [0, 64]");
    if (p->precision != KNNG_FP32 && p->precision != KNNG_BF16_SCREEN) return fail(KNNG_EINVAL, "unknown precision");
    if (p->path < KNNG_PATH_AUTO || p->path > KNNG_PATH_MFMA_BF16X3) return fail(KNNG_EINVAL, "unknown path");
    if (p->reorder < 0 || p->reorder > KNNG_MAX_ITERS) return fail(KNNG_EINVAL, "reorder must be in [0, 64]");
    if (p->blocks < 0 || (int64_t)p->blocks > N) return fail(KNNG_EINVAL, "blocks must be in [0, N]");
    if (p->sampling != KNNG_SAMPLING_WEIGHTED && p->sampling != KNNG_SAMPLING_TURBO)
        return fail(KNNG_EINVAL, "unknown sampling rule");
    if (N * (int64_t)p->K >= (1LL << 31)) return fail(KNNG_EINVAL, "N*K must be < 2^31");
    return KNNG_OK;
}

// AUTO's join path, from the single-Gaussian sweeps (n = 16384, K = 20): the
// direct form on the VALU up to d = 48, the split-BF16 form from d = 56, for
// one-plane and three-plane data alike (with FP64 step accumulation on
// inexact data the FP32 tiles trail the split form at every d).
constexpr int kAutoMatrixMinD = 56;

knng_status make_plan(int64_t N, int32_t d, const knng_params* p, Plan& P, bool rowkey_ok = true) {
    knng_status s = validate(N, d, p);
    if (s != KNNG_OK) return s;
    const int K = p->K;
    P.C = sample_cap(K, p->rho);
    P.turbo = p->sampling == KNNG_SAMPLING_TURBO ? 1 : 0;
    int path = p->path;
    P.bf16 = p->precision == KNNG_BF16_SCREEN ? 1 : 0;
    // the exact integer form (int8 tiles) was withdrawn after a device fault
    // whose cause was never shown; the value stays reserved
    if (path == KNNG_PATH_MFMA_I8) return fail(KNNG_EINVAL, "the exact integer form is not available");
    if (P.bf16) {
        if (path == KNNG_PATH_VALU || path == KNNG_PATH_MFMA_BF16X3)
            return fail(KNNG_EINVAL, "the BF16-screened form runs on the FP32 MFMA path");
        path = KNNG_PATH_MFMA;
    }
    if (path == KNNG_PATH_AUTO) {
        path = (d >= kAutoMatrixMinD && 2 * P.C <= 64) ? (P.bf16 ? KNNG_PATH_MFMA : KNNG_PATH_MFMA_BF16X3)
                                                        : KNNG_PATH_VALU;
    }
    if ((path == KNNG_PATH_MFMA || path == KNNG_PATH_MFMA_BF16X3) && 2 * P.C > 64)
        return fail(KNNG_EINVAL, "MFMA path needs ceil(rho*K) <= 32");
    P.split = path == KNNG_PATH_MFMA_BF16X3 ? 1 : 0;
    P.path = path;
    P.reorder = p->reorder ? 1 : 0;
    P.dp = (int)(path != KNNG_PATH_VALU ? round_up(d, 32) : round_up(d, 4));
    if (path == KNNG_PATH_VALU) {
        Views tv{};
        tv.C = P.C;
        tv.dp = P.dp;
        if (!join_valu_fits(tv))
            return fail(KNNG_EINVAL, "VALU path: 2*C rows of d floats do not fit the LDS stage; use the MFMA path");
    }
    const int64_t C = P.C;
    P.pmax = 2 * N * (int64_t)K * (2 * C - 1);   // sum of the bucket bounds (knng_kernels.hip, bucket_lo)
    if (P.pmax >= 0xffffffffLL) return fail(KNNG_EINVAL, "proposal capacity exceeds 2^32 slots");
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (size_t)round_up((int64_t)bytes, 256);
        return o;
    };
    const size_t NK = (size_t)N * K;
    P.o_Xp = take((size_t)N * P.dp * 4);
    P.o_nrm = take((size_t)N * 4);
    P.o_nrm64 = path != KNNG_PATH_VALU ? take((size_t)N * 8) : 0;
    P.o_orig = take((size_t)N * 4);
    P.o_posof = take((size_t)N * 4);
    P.o_lkey = take(NK * 8);
    P.o_lpos = take(NK * 4);
    P.o_kth = take((size_t)N * 8);
    P.rowkey = rowkey_ok && path == KNNG_PATH_VALU && P.dp == 4 ? 1 : 0;
    if (P.rowkey) P.o_rk = take((size_t)N * sizeof(RowKey));
    P.o_cnt4 = take((size_t)N * 4 * 4);   // rdeg, rcur, cap, pcnt: one fill
    P.o_roff = take(((size_t)N + 1) * 4);
    P.o_rev = take(NK * 16);
    P.o_cand = take((size_t)N * 2 * C * 8);
    P.o_nn = take((size_t)N * 4);
    P.o_big = take((size_t)N * 4);
    P.o_hubs = take((size_t)N * 4);
    P.o_poff = take(((size_t)N + 1) * 4);
    P.o_pkey = take((size_t)P.pmax * 8);
    P.o_scan = take(scan_tmp_words((int)N) * 4);
    P.o_counters = take(kNumCounters * 8);
    P.o_partial = take(partial_words() * 8);
    if (P.bf16) {
        P.o_Xb = take((size_t)N * P.dp * 2);
        P.o_nb = take((size_t)N * 8);
        if (p->reorder) {
            P.o_Xb2 = take((size_t)N * P.dp * 2);
            P.o_nb2 = take((size_t)N * 8);
        }
    }
    if (P.split) {
        P.o_Xs = take((size_t)3 * N * P.dp * 2);
        if (p->reorder) P.o_Xs2 = take((size_t)3 * N * P.dp * 2);
    }
    if (p->reorder) {   // permutation scratch only when the permutation is on
        P.o_comp = take((size_t)N * 4);
        P.o_pdone = take((size_t)N);
        P.o_comp2 = take((size_t)N * 4);
        P.o_par = take((size_t)N * 4);
        P.o_lvl = take((size_t)N * 4);
        P.o_best = take((size_t)N * 8);
        P.o_size = take((size_t)N * 4);
        P.o_offs = take(((size_t)N + 1) * 4);
        P.o_cur = take((size_t)N * 4);
        P.o_newpos = take((size_t)N * 4);
        P.o_lkey2 = take(NK * 8);
        P.o_lpos2 = take(NK * 4);
        P.o_kth2 = take((size_t)N * 8);
        if (P.rowkey) P.o_rk2 = take((size_t)N * sizeof(RowKey));
        P.o_Xp2 = take((size_t)N * P.dp * 4);
        P.o_nrm2 = take((size_t)N * 4);
        P.o_nrm64_2 = path != KNNG_PATH_VALU ? take((size_t)N * 8) : 0;
        P.o_orig2 = take((size_t)N * 4);
    }
    // counting-sort reverse bucketing: super-buckets of 2^shift positions, at
    // most kRevMaxS of them, blocks of E entries (at most 1024 blocks). The
    // shift grows while a block's run into one super-bucket averages under 8
    // entries (128 B: shorter runs are written as partial lines) and at least
    // 256 super-buckets remain (one workgroup each in k_rev_bucket). Smaller
    // super-buckets keep the region each k_rev_bucket workgroup scatters into
    // small enough for its lines to fill in L2 (at 4M points and K = 15:
    // 2^9 positions, about 120 KB per workgroup, against 480 KB at 2^11).
    P.rev_S = 0;
    int64_t E = 4096;
    while ((int64_t)(NK + E - 1) / E > 1024) E *= 2;
    for (int sh = 8; sh <= kRevMaxShift; ++sh) {
        const int64_t S = (N + (1LL << sh) - 1) >> sh;
        const int64_t S2 = (N + (2LL << sh) - 1) >> (sh + 1);
        if (sh < kRevMaxShift && E < 8 * S && S2 >= 256) continue;
        if (S <= kRevMaxS) {
            P.rev_shift = sh;
            P.rev_S = (int)S;
            P.rev_E = (int)E;
            P.rev_B = (int)((NK + E - 1) / E);
            const size_t cells = (size_t)P.rev_S * P.rev_B;
            P.o_rev_h = take(cells * 4);
            P.o_rev_hs = take((cells + 1) * 4);
            P.o_rev_tmp = take(scan_tmp_words((int)cells) * 4);
            break;
        }
    }
    P.o_flag = take(64);
    P.total = off;
    return KNNG_OK;
}

Views carve(const Plan& P, int64_t N, int32_t d, int K, void* ws) {
    char* b = static_cast<char*>(ws);
    Views v{};
    v.N = (int)N;
    v.d = d;
    v.dp = P.dp;
    v.K = K;
    v.C = P.C;
    v.turbo = P.turbo;
    v.Xp = reinterpret_cast<float*>(b + P.o_Xp);
    v.nrm = reinterpret_cast<float*>(b + P.o_nrm);
    if (P.path != KNNG_PATH_VALU) v.nrm64 = reinterpret_cast<double*>(b + P.o_nrm64);
    v.orig = reinterpret_cast<int32_t*>(b + P.o_orig);
    v.posof = reinterpret_cast<int32_t*>(b + P.o_posof);
    v.lkey = reinterpret_cast<uint64_t*>(b + P.o_lkey);
    v.lpos = reinterpret_cast<uint32_t*>(b + P.o_lpos);
    v.kth = reinterpret_cast<uint64_t*>(b + P.o_kth);
    if (P.rowkey) v.rk = reinterpret_cast<RowKey*>(b + P.o_rk);
    uint32_t* c4 = reinterpret_cast<uint32_t*>(b + P.o_cnt4);
    v.rdeg = c4;
    v.rcur = c4 + N;
    v.cap = c4 + 2 * N;
    v.pcnt = c4 + 3 * N;
    v.roff = reinterpret_cast<uint32_t*>(b + P.o_roff);
    v.rev = reinterpret_cast<uint4*>(b + P.o_rev);
    v.cand = reinterpret_cast<uint2*>(b + P.o_cand);
    v.nn = reinterpret_cast<uint32_t*>(b + P.o_nn);
    v.big = reinterpret_cast<uint32_t*>(b + P.o_big);
    v.hubs = reinterpret_cast<uint32_t*>(b + P.o_hubs);
    v.poff = reinterpret_cast<uint32_t*>(b + P.o_poff);
    v.pkey = reinterpret_cast<uint64_t*>(b + P.o_pkey);
    v.scan_tmp = reinterpret_cast<uint32_t*>(b + P.o_scan);
    v.counters = reinterpret_cast<uint64_t*>(b + P.o_counters);
    v.partial = reinterpret_cast<uint64_t*>(b + P.o_partial);
    if (P.bf16) {
        v.Xb = reinterpret_cast<uint16_t*>(b + P.o_Xb);
        v.nb = reinterpret_cast<float2*>(b + P.o_nb);
        if (P.reorder) {
            v.Xb2 = reinterpret_cast<uint16_t*>(b + P.o_Xb2);
            v.nb2 = reinterpret_cast<float2*>(b + P.o_nb2);
        }
    }
    if (P.reorder) {
        v.comp = reinterpret_cast<int32_t*>(b + P.o_comp);
        v.pdone = reinterpret_cast<uint8_t*>(b + P.o_pdone);
        v.comp2 = reinterpret_cast<int32_t*>(b + P.o_comp2);
        v.par = reinterpret_cast<int32_t*>(b + P.o_par);
        v.lvl = reinterpret_cast<uint32_t*>(b + P.o_lvl);
        v.best = reinterpret_cast<uint64_t*>(b + P.o_best);
        v.size = reinterpret_cast<uint32_t*>(b + P.o_size);
        v.offs = reinterpret_cast<uint32_t*>(b + P.o_offs);
        v.cur = reinterpret_cast<uint32_t*>(b + P.o_cur);
        v.newpos = reinterpret_cast<int32_t*>(b + P.o_newpos);
        v.lkey2 = reinterpret_cast<uint64_t*>(b + P.o_lkey2);
        v.lpos2 = reinterpret_cast<uint32_t*>(b + P.o_lpos2);
        v.kth2 = reinterpret_cast<uint64_t*>(b + P.o_kth2);
        if (P.rowkey) v.rk2 = reinterpret_cast<RowKey*>(b + P.o_rk2);
        v.Xp2 = reinterpret_cast<float*>(b + P.o_Xp2);
        v.nrm2 = reinterpret_cast<float*>(b + P.o_nrm2);
        if (P.path != KNNG_PATH_VALU) v.nrm64_2 = reinterpret_cast<double*>(b + P.o_nrm64_2);
        v.orig2 = reinterpret_cast<int32_t*>(b + P.o_orig2);
    }
    v.planes = 3;   // until the create-time count (single builds)
    if (P.split) {
        v.Xs = reinterpret_cast<uint16_t*>(b + P.o_Xs);
        if (P.reorder) v.Xs2 = reinterpret_cast<uint16_t*>(b + P.o_Xs2);
    }
    if (P.rev_S) {
        v.rev_shift = P.rev_shift;
        v.rev_S = P.rev_S;
        v.rev_B = P.rev_B;
        v.rev_E = P.rev_E;
        v.rev_h = reinterpret_cast<uint32_t*>(b + P.o_rev_h);
        v.rev_hs = reinterpret_cast<uint32_t*>(b + P.o_rev_hs);
        v.rev_tmp = reinterpret_cast<uint32_t*>(b + P.o_rev_tmp);
    }
    v.flag = reinterpret_cast<uint32_t*>(b + P.o_flag);
    return v;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(KNNG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

}  // namespace

constexpr int kNumEvents = 13;

struct knng_ctx {
    Views v;
    Plan plan;
    knng_params p;
    int64_t N;
    int32_t d;
    hipStream_t stream;
    const float* dX;
    void* ws;
    int t;               // iterations completed
    bool permuted;
    int perm_levels;
    bool has_graph;
    knng_stats stats;
    hipEvent_t ev[kNumEvents];   // phase events of odd (0..3) and even (6..9) iterations; 4, 5: permutation;
                                 // 10..12: start, end of init, end of the build
    uint64_t hc[kNumCounters];
    uint64_t* hslot;     // pinned: the counters of iteration t at hslot[t * kNumCounters]
    uint64_t* dslot;     // the same memory as the device addresses it (allocation-free
                         // build: device slots in the static scratch, no host mapping)
    bool noalloc;        // allocation-free build: no events, no pinned slots, no timings
};

namespace {

// Pinned counter slots (a few KB each, mapped into the device's address
// space), kept for reuse across contexts so a build pays no host allocation.
constexpr size_t kSlotBytes = (size_t)(KNNG_MAX_ITERS + 1) * kNumCounters * sizeof(uint64_t);
std::mutex g_slot_mu;
std::vector<std::pair<uint64_t*, uint64_t*>> g_slot_free;   // {host, device}

bool slot_take(uint64_t** host, uint64_t** dev) {
    {
        std::lock_guard<std::mutex> lk(g_slot_mu);
        if (!g_slot_free.empty()) {
            *host = g_slot_free.back().first;
            *dev = g_slot_free.back().second;
            g_slot_free.pop_back();
            return true;
        }
    }
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, kSlotBytes, hipHostMallocMapped) != hipSuccess) return false;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || !d) {
        (void)hipHostFree(h);
        return false;
    }
    std::memset(h, 0, kSlotBytes);
    *host = static_cast<uint64_t*>(h);
    *dev = static_cast<uint64_t*>(d);
    return true;
}

void slot_give(uint64_t* host, uint64_t* dev) {
    std::lock_guard<std::mutex> lk(g_slot_mu);
    g_slot_free.emplace_back(host, dev);
}

// Phase events, kept for reuse across contexts like the slots (per device:
// an event records only on streams of the device it was created on).
std::mutex g_ev_mu;
std::vector<std::pair<int, std::array<hipEvent_t, kNumEvents>>> g_ev_free;   // {device, events}

bool events_take(hipEvent_t (&ev)[kNumEvents]) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        for (size_t i = g_ev_free.size(); i-- > 0;) {
            if (g_ev_free[i].first != dev) continue;
            for (int k = 0; k < kNumEvents; ++k) ev[k] = g_ev_free[i].second[k];
            g_ev_free.erase(g_ev_free.begin() + (std::ptrdiff_t)i);
            return true;
        }
    }
    for (auto& e : ev) e = nullptr;
    for (auto& e : ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            for (auto& f : ev)
                if (f) (void)hipEventDestroy(f);
            for (auto& f : ev) f = nullptr;
            return false;
        }
    }
    return true;
}

void events_give(hipEvent_t (&ev)[kNumEvents]) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    } else {
        std::array<hipEvent_t, kNumEvents> a;
        for (int k = 0; k < kNumEvents; ++k) a[k] = ev[k];
        std::lock_guard<std::mutex> lk(g_ev_mu);
        g_ev_free.emplace_back(dev, a);
    }
    for (auto& e : ev) e = nullptr;
}

knng_status read_counters(knng_ctx* c) {
    HIP_TRY(hipMemcpyAsync(c->hc, c->v.counters, sizeof(c->hc), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return KNNG_OK;
}

float ms_between(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.f;
    return ms;
}

// Graph-ordered permutation (Sec. 3.2), once after iteration 1: cluster the
// current lists level by level (a read-back every 4 levels to stop early),
// lay the hook forest out, move rows and lists, and swap the buffers.
knng_status do_permute(knng_ctx* c) {
    Views& v = c->v;
    hipStream_t s = c->stream;
    if (!c->noalloc) HIP_TRY(hipEventRecord(c->ev[4], s));
    launch_perm_begin(v, s);
    uint32_t fl[4] = {0, 0, 0, 0};
    for (int l = 0; l < perm_levels_max(); l += 4) {
        for (int j = 0; j < 4; ++j) launch_perm_level(v, (uint32_t)(l + j), s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(fl, v.flag, sizeof(fl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (fl[0]) break;
    }
    launch_perm_finish(v, fl[2], s);
    std::swap(v.Xp, v.Xp2);
    std::swap(v.nrm, v.nrm2);
    std::swap(v.nrm64, v.nrm64_2);
    std::swap(v.orig, v.orig2);
    std::swap(v.lkey, v.lkey2);
    std::swap(v.lpos, v.lpos2);
    std::swap(v.kth, v.kth2);
    std::swap(v.rk, v.rk2);
    std::swap(v.Xb, v.Xb2);
    std::swap(v.nb, v.nb2);
    if (v.Xs) std::swap(v.Xs, v.Xs2);
    launch_perm_posof(v, s);
    v.permuted = 1;
    if (!c->noalloc) HIP_TRY(hipEventRecord(c->ev[5], s));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    c->stats.reorder_ms = c->noalloc ? 0.f : ms_between(c->ev[4], c->ev[5]);
    c->perm_levels = (int)fl[2];
    knng_status rs = read_counters(c);
    if (rs != KNNG_OK) return rs;
    if (c->hc[kCntError]) {
        char buf[96];
        snprintf(buf, sizeof buf, "device invariant failed in the permutation (code %llu)",
                 (unsigned long long)c->hc[kCntError]);
        return fail(KNNG_EDEVICE, buf);
    }
    c->permuted = true;
    return KNNG_OK;
}

hipEvent_t* phase_events(knng_ctx* c, int t) { return (t & 1) ? &c->ev[0] : &c->ev[6]; }

// Enqueues iteration t (sampling, join, merge). thr >= 0: the device records
// whether the stop rule held (changes < thr) so that an iteration enqueued
// ahead of the host's decision returns at once.
// Block-asynchronous iterations (params.blocks = B > 1) enqueue B rounds of
// the same steps: round b samples and joins only the owners with original
// ids in [N b / B, N (b + 1) / B) from the graph the earlier rounds left, and
// its merge updates every list before round b + 1 samples; the counters add
// up over the rounds. Phase events: sampling from the first round's start,
// the last round's join and merge.
knng_status enqueue_iteration(knng_ctx* c, int t, double thr) {
    const Views& v = c->v;
    hipStream_t s = c->stream;
    hipEvent_t* E = phase_events(c, t);
    const uint64_t st = stream_state(c->p.seed, 2, (uint64_t)t);
    const int B = c->p.blocks > 1 ? c->p.blocks : 1;
    for (int b = 0; b < B; ++b) {
        const bool first = b == 0, last = b == B - 1;
        Views vb = v;
        if (B > 1) {
            vb.blk_on = 1;
            vb.blk_lo = (int)((int64_t)v.N * b / B);
            vb.blk_hi = (int)((int64_t)v.N * (b + 1) / B);
        }
        // counters and proposal-bucket cursors are cleared by the previous merge
        // (and at create); the atomic reverse path counts into rdeg and rcur
        if (!v.rev_S) launch_fill_u32(v.rdeg, 0u, 2 * (int64_t)v.N, s);
        // phase events: start of sampling (E0), start / end of the join (E1,
        // E2), end of the merge (E3), stamped by the dispatches themselves
        hipEvent_t e0 = first ? E[0] : nullptr, e1 = last ? E[1] : nullptr, e2 = last ? E[2] : nullptr;
        if (v.rev_S) {
            launch_rev_partition(v, st, t, s, e0);
        } else {
            launch_rev_hist(v, s, e0);
            launch_scan(v.rdeg, v.roff, v.N, v.scan_tmp, s);
            launch_rev_scatter(v, st, t, s);
        }
        launch_select(vb, st, t, s);
        if (c->plan.bf16)
            launch_join_bf16(vb, s, e1, e2);
        else if (c->plan.path == KNNG_PATH_MFMA_BF16X3)
            launch_join_split(vb, s, e1, e2);
        else if (c->plan.path == KNNG_PATH_MFMA)
            launch_join_mfma(vb, s, e1, e2);
        else
            launch_join_valu(vb, s, e1, e2);
        launch_merge(v, s);
        launch_finish_counters(v, s, last ? E[3] : nullptr, c->dslot + (size_t)t * kNumCounters, thr, last ? 1 : 0);
    }
    HIP_TRY(hipGetLastError());
    return KNNG_OK;
}

// Waits for iteration t (enqueued last but possibly one) and records its
// statistics.
knng_status finish_iteration(knng_ctx* c, int t, int64_t* evals, int64_t* changes) {
    hipEvent_t* E = phase_events(c, t);
    if (c->noalloc) {
        HIP_TRY(hipMemcpyAsync(c->hc, c->dslot + (size_t)t * kNumCounters, sizeof(c->hc), hipMemcpyDeviceToHost,
                               c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    } else {
        HIP_TRY(hipEventSynchronize(E[3]));
        std::memcpy(c->hc, c->hslot + (size_t)t * kNumCounters, sizeof(c->hc));
    }
    if (c->hc[kCntError]) {
        char buf[96];
        snprintf(buf, sizeof buf, "device invariant failed in iteration %d (code %llu)", t,
                 (unsigned long long)c->hc[kCntError]);
        return fail(KNNG_EDEVICE, buf);
    }
    const int64_t e = (int64_t)(c->hc[kCntPairs2] / 2);
    const int64_t ch = (int64_t)c->hc[kCntChanges];
    knng_stats& S = c->stats;
    const int i = t - 1;
    S.evals[i] = e;
    S.changes[i] = ch;
    S.proposals[i] = (int64_t)c->hc[kCntProposals];
    S.rescored[i] = (int64_t)c->hc[kCntRescored];
    if (!c->noalloc) {
        S.sample_ms[i] = ms_between(E[0], E[1]);
        S.join_ms[i] = ms_between(E[1], E[2]);
        S.merge_ms[i] = ms_between(E[2], E[3]);
        S.iter_ms[i] = ms_between(E[0], E[3]);
    }
    S.iters = t;
    c->t = t;
    if (evals) *evals = e;
    if (changes) *changes = ch;
    return KNNG_OK;
}

// params.reorder = t_p >= 1: the permutation runs once, after iteration t_p
bool permute_after(const knng_ctx* c, int t) { return c->p.reorder > 0 && t == c->p.reorder && !c->permuted; }

// One iteration, host-driven (step API): no look-ahead.
knng_status do_iterate(knng_ctx* c, int64_t* evals, int64_t* changes) {
    if (!c->has_graph) return fail(KNNG_EINVAL, "no graph: call knng_init_graph or knng_load_graph first");
    if (c->t >= KNNG_MAX_ITERS) return fail(KNNG_EINVAL, "iteration limit of the statistics reached");
    const int t = c->t + 1;
    knng_status st = enqueue_iteration(c, t, -1.0);
    if (st != KNNG_OK) return st;
    st = finish_iteration(c, t, evals, changes);
    if (st != KNNG_OK) return st;
    if (permute_after(c, t)) return do_permute(c);
    return KNNG_OK;
}

int dist_mode(const knng_ctx* c) {
    if (c->plan.path == KNNG_PATH_MFMA_BF16X3) return kDistGram;
    return (c->plan.path == KNNG_PATH_MFMA && !c->plan.bf16) ? kDistGram : kDistDirect;
}

}  // namespace

namespace {

// The allocation-free build's workspace: a static device array that every
// device the library runs on holds for the life of the process. In host code
// `scratch` names a host-side stand-in, never a device address: the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current.
constexpr size_t kScratchBytes = (size_t)KNNG_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

knng_status scratch_base(char** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(KNNG_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(KNNG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<char*>(p);
    }
    *out = g_scratch[dev];
    return KNNG_OK;
}

// init, iterations until the stop rule or max_iters, write-out (the body of
// both build entry points). Events only when the context has them.
knng_status run_build(knng_ctx* c, const knng_params* params, int32_t* d_ids, float* d_dists, knng_stats* stats) {
    hipEvent_t e0 = c->noalloc ? nullptr : c->ev[10];
    hipEvent_t e1 = c->noalloc ? nullptr : c->ev[11];
    hipEvent_t e2 = c->noalloc ? nullptr : c->ev[12];
    auto done = [](knng_status st) { return st; };
    if (e0) (void)hipEventRecord(e0, c->stream);
    knng_status s = knng_init_graph(c);
    if (s != KNNG_OK) return done(s);
    if (e1) (void)hipEventRecord(e1, c->stream);
    const int64_t N = c->N;
    const double thr = (double)params->delta * (double)N * (double)params->K;
    const int T = std::min(params->max_iters, KNNG_MAX_ITERS);
    bool conv = false;
    // One iteration ahead: iteration t + 1 is enqueued before the host reads
    // iteration t's counters, and returns at once on the device if t met the
    // stop rule (the same test, c_t < delta N K, on both sides). Not across
    // the permutation.
    if (T > 0 && (s = enqueue_iteration(c, 1, thr)) != KNNG_OK) return done(s);
    for (int t = 1; t <= T; ++t) {
        const bool ahead = t < T && !permute_after(c, t);
        if (ahead && (s = enqueue_iteration(c, t + 1, thr)) != KNNG_OK) return done(s);
        int64_t e = 0, ch = 0;
        s = finish_iteration(c, t, &e, &ch);
        if (s == KNNG_OK && permute_after(c, t)) s = do_permute(c);
        if (s != KNNG_OK) return done(s);
        if ((double)ch < thr) {
            conv = true;
            break;
        }
        if (!ahead && t < T && (s = enqueue_iteration(c, t + 1, thr)) != KNNG_OK) return done(s);
    }
    launch_finalize(c->v, d_ids, d_dists, nullptr, c->stream);
    if (e2) (void)hipEventRecord(e2, c->stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
        return done(fail(KNNG_EDEVICE, "finalize failed"));
    c->stats.converged = conv ? 1 : 0;
    if (e0) {
        c->stats.init_ms = ms_between(e0, e1);
        c->stats.total_ms = ms_between(e0, e2);
        float acc = c->stats.init_ms + c->stats.reorder_ms;
        for (int i = 0; i < c->stats.iters; ++i) acc += c->stats.iter_ms[i];
        c->stats.finalize_ms = c->stats.total_ms - acc > 0.f ? c->stats.total_ms - acc : 0.f;
    }
    if (stats) *stats = c->stats;
    return done((conv || params->max_iters == 0) ? KNNG_OK : KNNG_ENOTCONV);
}

}  // namespace

extern "C" {

const char* knng_last_error(void) { return g_err.c_str(); }

int32_t knng_sample_cap(int32_t K, double rho) { return sample_cap(K, rho); }

size_t knng_workspace_bytes(int64_t N, int32_t d, const knng_params* params) {
    Plan P{};
    if (make_plan(N, d, params, P) != KNNG_OK) return 0;
    return P.total;
}

}  // extern "C"

namespace {

// Binds a context to its inputs and workspace, lays the rows out and checks
// X (one synchronisation). dev_slots == nullptr: phase events and pinned
// counter slots; else the allocation-free form (counter slots in device
// memory, no events).
knng_status ctx_init(knng_ctx* c, const Plan& P, const float* dX, int64_t N, int32_t d, const knng_params* params,
                     void* d_ws, void* stream, uint64_t* dev_slots) {
    c->plan = P;
    c->p = *params;
    c->N = N;
    c->d = d;
    c->stream = static_cast<hipStream_t>(stream);
    c->dX = dX;
    c->ws = d_ws;
    c->v = carve(P, N, d, params->K, d_ws);
    std::memset(&c->stats, 0, sizeof(c->stats));
    c->stats.path = P.path;
    c->stats.precision = P.bf16 ? KNNG_BF16_SCREEN : KNNG_FP32;
    c->stats.dpad = P.dp;
    if (dev_slots) {
        c->noalloc = true;
        c->dslot = dev_slots;
    } else {
        if (!events_take(c->ev)) return fail(KNNG_EDEVICE, "hipEventCreate failed");
        if (!slot_take(&c->hslot, &c->dslot))
            return fail(KNNG_EDEVICE, "pinned counter slots: hipHostMalloc failed");
    }
    c->v.stop = c->v.flag + kStopFlag;
    launch_fill_u64(c->v.counters, 0ull, kNumCounters, c->stream);
    launch_fill_u32(c->v.nn, 0u, N, c->stream);   // no owner has a sample before its first iteration
    launch_fill_u32(c->v.pcnt, 0u, N, c->stream);
    launch_fill_u32(c->v.stop, 0u, 1, c->stream);
    if (P.path == KNNG_PATH_VALU) {
        launch_pad_rows(dX, c->v, c->stream);
    } else {
        launch_prep(dX, c->v, P.split, c->stream);
    }
    if (P.bf16) launch_make_bf16(c->v, c->stream);
    if (hipGetLastError() != hipSuccess || read_counters(c) != KNNG_OK) return fail(KNNG_EDEVICE, "row padding failed");
    if (c->hc[kCntNonFinite]) return fail(KNNG_EINVAL, "X holds a NaN or an infinity");
    if (P.path != KNNG_PATH_VALU && !P.bf16) {
        // FP32 Gram sums are exact only for integers with squared norms <= 2^23
        c->v.acc = (c->hc[kCntSplit] & kLayoutInexact) ? 1 : 0;
        c->stats.accurate = c->v.acc;
    }
    if (P.split) {
        const uint64_t used = c->hc[kCntSplit];
        c->v.planes = (used & 2u) ? 3 : (used & 1u) ? 2 : 1;
        c->stats.planes = c->v.planes;
        // 8-bit data: integers in 0..255 with exact FP32 sums read as byte rows
        c->v.u8 = c->v.planes == 1 && !c->v.acc && !(used & 16u) ? 1 : 0;
        c->stats.u8 = c->v.u8;
        if (c->v.planes > 1) launch_prep_rest(dX, c->v, c->stream);
    }
    c->stats.path = c->plan.path;
    return KNNG_OK;
}

// Returns what ctx_init took: pinned slots and events (after the stream has
// drained), to the pools.
void ctx_release(knng_ctx* c) {
    if (c->hslot || c->ev[0]) (void)hipStreamSynchronize(c->stream);   // no kernel writes the slots or records the events any more
    if (c->hslot) {
        slot_give(c->hslot, c->dslot);
        c->hslot = nullptr;
    }
    if (c->ev[0]) events_give(c->ev);
}

}  // namespace

extern "C" {

knng_status knng_create(knng_ctx** out, const float* dX, int64_t N, int32_t d, const knng_params* params,
                        void* d_ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!out) return fail(KNNG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dX) return fail(KNNG_EINVAL, "dX is NULL");
    if (!d_ws) return fail(KNNG_EINVAL, "workspace is NULL");
    Plan P{};
    knng_status s = make_plan(N, d, params, P);
    if (s != KNNG_OK) return s;
    if (ws_bytes < P.total) {
        char buf[128];
        snprintf(buf, sizeof buf, "workspace too small: %zu < %zu bytes", ws_bytes, P.total);
        return fail(KNNG_ENOMEM, buf);
    }
    knng_ctx* c = new (std::nothrow) knng_ctx();
    if (!c) return fail(KNNG_ENOMEM, "host allocation of the context failed");
    s = ctx_init(c, P, dX, N, d, params, d_ws, stream, nullptr);
    if (s != KNNG_OK) {
        knng_destroy(c);
        return s;
    }
    *out = c;
    return KNNG_OK;
}

knng_status knng_init_graph(knng_ctx* c) {
    if (!c) return fail(KNNG_EINVAL, "ctx is NULL");
    if (c->permuted) return fail(KNNG_EINVAL, "init after permutation is not supported");
    launch_fill_u32(c->v.stop, 0u, 1, c->stream);
    launch_init(c->v, stream_state(c->p.seed, 1, 0), dist_mode(c), c->stream);
    HIP_TRY(hipGetLastError());
    c->t = 0;
    c->has_graph = true;
    return KNNG_OK;
}

knng_status knng_load_graph(knng_ctx* c, const int32_t* d_ids, const float* d_dists, const uint8_t* d_flags,
                            int32_t t) {
    if (!c) return fail(KNNG_EINVAL, "ctx is NULL");
    if (!d_ids || !d_flags) return fail(KNNG_EINVAL, "ids/flags are NULL");
    if (c->permuted) return fail(KNNG_EINVAL, "load after permutation is not supported");
    if (t < 0 || t >= KNNG_MAX_ITERS) return fail(KNNG_EINVAL, "t out of range");
    launch_fill_u64(c->v.counters, 0ull, kNumCounters, c->stream);
    launch_fill_u32(c->v.stop, 0u, 1, c->stream);
    launch_load_rows(c->v, d_ids, d_dists, d_flags, dist_mode(c), c->stream);
    HIP_TRY(hipGetLastError());
    knng_status rs = read_counters(c);
    if (rs != KNNG_OK) return rs;
    if (c->hc[kCntError]) {
        c->has_graph = false;
        return fail(KNNG_EINVAL, "loaded rows must hold K distinct ids in [0, N) other than the row's own");
    }
    c->t = t;
    c->has_graph = true;
    return KNNG_OK;
}

knng_status knng_iterate(knng_ctx* c, int64_t* evals, int64_t* changes) {
    if (!c) return fail(KNNG_EINVAL, "ctx is NULL");
    return do_iterate(c, evals, changes);
}

knng_status knng_export(knng_ctx* c, int32_t* d_ids, float* d_dists, uint8_t* d_flags) {
    if (!c) return fail(KNNG_EINVAL, "ctx is NULL");
    if (!c->has_graph) return fail(KNNG_EINVAL, "no graph");
    if (!d_ids && !d_dists && !d_flags) return fail(KNNG_EINVAL, "no output given");
    launch_finalize(c->v, d_ids, d_dists, d_flags, c->stream);
    HIP_TRY(hipGetLastError());
    return KNNG_OK;
}

knng_status knng_export_samples(knng_ctx* c, int32_t* d_new, int32_t* d_old, int32_t* d_counts) {
    if (!c) return fail(KNNG_EINVAL, "ctx is NULL");
    if (!d_new || !d_old || !d_counts) return fail(KNNG_EINVAL, "outputs are NULL");
    if (c->t < 1) return fail(KNNG_EINVAL, "no iteration has run");
    launch_export_samples(c->v, d_new, d_old, d_counts, c->stream);
    HIP_TRY(hipGetLastError());
    return KNNG_OK;
}

knng_status knng_export_order(knng_ctx* c, int32_t* d_orig_of_pos) {
    if (!c || !d_orig_of_pos) return fail(KNNG_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(d_orig_of_pos, c->v.orig, sizeof(int32_t) * (size_t)c->N, hipMemcpyDeviceToDevice,
                           c->stream));
    return KNNG_OK;
}

knng_status knng_get_stats(const knng_ctx* c, knng_stats* stats) {
    if (!c || !stats) return fail(KNNG_EINVAL, "NULL argument");
    *stats = c->stats;
    return KNNG_OK;
}

void knng_destroy(knng_ctx* c) {
    if (!c) return;
    ctx_release(c);
    delete c;
}

knng_status knng_build(const float* dX, int64_t N, int32_t d, const knng_params* params, int32_t* d_ids,
                       float* d_dists, void* d_ws, size_t ws_bytes, void* stream, knng_stats* stats) {
    if (!d_ids || !d_dists) return fail(KNNG_EINVAL, "outputs are NULL");
    knng_ctx* c = nullptr;
    knng_status s = knng_create(&c, dX, N, d, params, d_ws, ws_bytes, stream);
    if (s != KNNG_OK) return s;
    s = run_build(c, params, d_ids, d_dists, stats);
    knng_destroy(c);
    return s;
}

knng_status knng_build_noalloc(const float* dX, int64_t N, int32_t d, const knng_params* params, int32_t* d_ids,
                               float* d_dists, void* stream, knng_stats* stats) {
    g_err.clear();
    if (!dX) return fail(KNNG_EINVAL, "dX is NULL");
    if (!d_ids || !d_dists) return fail(KNNG_EINVAL, "outputs are NULL");
    Plan P{};
    knng_status s = make_plan(N, d, params, P);
    if (s != KNNG_OK) return s;
    const size_t need = P.total + kSlotBytes;   // workspace, then the counter slots
    if (need > kScratchBytes) {
        char buf[192];
        snprintf(buf, sizeof buf,
                 "allocation-free build needs %zu bytes of scratch; the static scratch holds %zu "
                 "(use knng_build with a workspace)", need, kScratchBytes);
        return fail(KNNG_ENOMEM, buf);
    }
    char* base = nullptr;
    s = scratch_base(&base);
    if (s != KNNG_OK) return s;
    knng_ctx c{};   // on the stack: nothing is allocated
    s = ctx_init(&c, P, dX, N, d, params, base, stream, reinterpret_cast<uint64_t*>(base + P.total));
    if (s == KNNG_OK) s = run_build(&c, params, d_ids, d_dists, stats);
    ctx_release(&c);
    return s;
}

}  // extern "C"
// ====================================================================== batched form
//
// Datasets with the same padded row length and join path form one group; a
// group is one union build (contiguous position range per dataset, per-dataset
// seeds, iteration counters, stop rules and statistics on the device). The
// execute call only enqueues kernels (no allocation, no synchronisation), so
// it can be captured in a graph; all groups and all T_max iterations form one
// graph launch. Finished datasets are skipped by every kernel.

namespace {

struct BatchGroup {
    int d = 0, dp = 0, path = 0;
    int cap = 0;                // workgroup cap of the select and join passes (0: per owner group)
    std::vector<int> members;   // dataset indices in the caller's order
    int64_t N = 0;
    Plan plan{};
    size_t off = 0;             // byte offset of the group's region in the workspace
    size_t tables_off = 0;      // offset of the batch tables inside the region
    Views v{};
};

struct TableLayout {
    size_t ds, dsbase, active, st_init, st_table, chg, chgoff, out_ids, out_dists, in_X, in_d, iters, conv, stats, total;
};

TableLayout table_layout(int64_t N, int nds, int T) {
    TableLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (size_t)round_up((int64_t)bytes, 256);
        return o;
    };
    L.ds = take((size_t)N * 4);
    L.dsbase = take(((size_t)nds + 1) * 4);
    L.active = take((size_t)nds * 4);
    L.st_init = take((size_t)nds * 8);
    L.st_table = take((size_t)nds * T * 8);
    L.chg = take((size_t)N * 4);
    L.chgoff = take(((size_t)N + 1) * 4);
    L.out_ids = take((size_t)nds * 8);
    L.out_dists = take((size_t)nds * 8);
    L.in_X = take((size_t)nds * 8);
    L.in_d = take((size_t)nds * 4);
    L.iters = take((size_t)nds * 4);
    L.conv = take((size_t)nds * 4);
    L.stats = take((size_t)nds * T * 16);
    L.total = off;
    return L;
}

// "16:valu,64:mfma@2048" -> {path, workgroup cap} for d; path 0 if d is absent
struct Tuned {
    int path = 0, cap = 0;
};

Tuned parse_tuned(const std::string& table, int d) {
    size_t pos = 0;
    while (pos < table.size()) {
        size_t end = table.find(',', pos);
        if (end == std::string::npos) end = table.size();
        const std::string item = table.substr(pos, end - pos);
        const size_t c = item.find(':');
        if (c != std::string::npos && std::atoi(item.substr(0, c).c_str()) == d) {
            std::string v = item.substr(c + 1);
            Tuned t;
            const size_t at = v.find('@');
            if (at != std::string::npos) {
                t.cap = std::max(0, std::atoi(v.substr(at + 1).c_str()));
                v = v.substr(0, at);
            }
            if (v == "valu") t.path = KNNG_PATH_VALU;
            if (v == "mfma") t.path = KNNG_PATH_MFMA;
            if (v == "bf16x3") t.path = KNNG_PATH_MFMA_BF16X3;
            if (t.path) return t;
        }
        pos = end + 1;
    }
    return Tuned{};
}

std::string tuned_entry(int d, int path, int cap) {
    std::string e = std::to_string(d) + (path == KNNG_PATH_MFMA ? ":mfma" : path == KNNG_PATH_MFMA_BF16X3 ? ":bf16x3" : ":valu");
    if (cap > 0) e += "@" + std::to_string(cap);
    return e;
}

}  // namespace

struct knng_batch {
    knng_params p{};
    std::vector<knng_dataset> descs;
    std::vector<BatchGroup> groups;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    std::string tuning;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

knng_status batch_validate(const knng_dataset* descs, int32_t n, const knng_params* p) {
    if (!descs || n < 1) return fail(KNNG_EINVAL, "no datasets");
    if (!p) return fail(KNNG_EINVAL, "params is NULL");
    if (p->reorder) return fail(KNNG_EINVAL, "the batched form runs without the permutation");
    if (p->blocks > 1) return fail(KNNG_EINVAL, "the batched form runs synchronous iterations");
    if (p->precision != KNNG_FP32) return fail(KNNG_EINVAL, "the batched form runs in FP32");
    if (p->max_iters < 1) return fail(KNNG_EINVAL, "the batched form needs max_iters >= 1");
    for (int i = 0; i < n; ++i) {
        if (!descs[i].dX || !descs[i].d_ids || !descs[i].d_dists) return fail(KNNG_EINVAL, "dataset pointer is NULL");
        knng_status s = validate(descs[i].N, descs[i].d, p);
        if (s != KNNG_OK) return s;
    }
    return KNNG_OK;
}

// groups by (padded length, path); the path per d comes from the tuning table
// or defaults to the single-build rule
knng_status batch_groups(const knng_dataset* descs, int32_t n, const knng_params* p, const std::string& tuning,
                         std::vector<BatchGroup>& groups, size_t& total) {
    groups.clear();
    const int C = sample_cap(p->K, p->rho);
    for (int i = 0; i < n; ++i) {
        const int d = descs[i].d;
        const Tuned tu = parse_tuned(tuning, d);
        int path = p->path != KNNG_PATH_AUTO ? p->path : tu.path;
        if (!path) path = (d >= kAutoMatrixMinD && 2 * C <= 64) ? KNNG_PATH_MFMA_BF16X3 : KNNG_PATH_VALU;
        const int dp = (int)(path != KNNG_PATH_VALU ? round_up(d, 32) : round_up(d, 4));
        BatchGroup* g = nullptr;
        for (auto& x : groups)
            if (x.dp == dp && x.path == path && x.d == d) g = &x;
        if (!g) {
            groups.push_back(BatchGroup{});
            g = &groups.back();
            g->d = d;
            g->dp = dp;
            g->path = path;
            g->cap = tu.cap;
        }
        g->members.push_back(i);
        g->N += descs[i].N;
    }
    total = 0;
    for (auto& g : groups) {
        if (g.N >= (1LL << 31) / p->K) return fail(KNNG_EINVAL, "a dimension group is too large for one union");
        knng_params gp = *p;
        gp.path = g.path;
        gp.reorder = 0;
        Plan P{};
        knng_status s = make_plan(g.N, g.d, &gp, P, false);   // batch setup lays out Xp rows only
        if (s != KNNG_OK) return s;
        g.plan = P;
        g.off = total;
        g.tables_off = P.total;
        total += P.total + table_layout(g.N, (int)g.members.size(), p->max_iters).total;
        total = (size_t)round_up((int64_t)total, 4096);
    }
    return KNNG_OK;
}

knng_status batch_upload(knng_batch* b, hipStream_t s) {
    const int T = b->p.max_iters;
    for (auto& g : b->groups) {
        const int nds = (int)g.members.size();
        const TableLayout L = table_layout(g.N, nds, T);
        char* base = b->ws + g.off;
        g.v = carve(g.plan, g.N, g.d, b->p.K, base);
        char* tb = base + g.tables_off;
        Views& v = g.v;
        // matrix paths: FP64 accumulation for every group (on data whose FP32
        // sums are exact it gives the same values as FP32, so every dataset
        // matches its single build either way)
        v.acc = g.path != KNNG_PATH_VALU ? 1 : 0;
        v.stop = v.flag + kStopFlag;   // set once every dataset of the group has stopped
        v.grid_cap = g.cap;
        v.nds = nds;
        v.ds = reinterpret_cast<uint32_t*>(tb + L.ds);
        v.dsbase = reinterpret_cast<uint32_t*>(tb + L.dsbase);
        v.active = reinterpret_cast<uint32_t*>(tb + L.active);
        v.st_init = reinterpret_cast<uint64_t*>(tb + L.st_init);
        v.st_table = reinterpret_cast<uint64_t*>(tb + L.st_table);
        v.chg = reinterpret_cast<uint32_t*>(tb + L.chg);
        v.chgoff = reinterpret_cast<uint32_t*>(tb + L.chgoff);
        v.out_ids = reinterpret_cast<int32_t* const*>(tb + L.out_ids);
        v.out_dists = reinterpret_cast<float* const*>(tb + L.out_dists);
        v.in_X = reinterpret_cast<const float* const*>(tb + L.in_X);
        v.in_d = reinterpret_cast<int32_t*>(tb + L.in_d);
        v.ds_iters = reinterpret_cast<int32_t*>(tb + L.iters);
        v.ds_conv = reinterpret_cast<int32_t*>(tb + L.conv);
        v.ds_stats = reinterpret_cast<int64_t*>(tb + L.stats);
        std::vector<uint32_t> dsbase(nds + 1);
        std::vector<uint64_t> st_init(nds), st_table((size_t)nds * T);
        std::vector<const void*> oi(nds), od(nds), ix(nds);
        std::vector<int32_t> idd(nds);
        uint32_t acc = 0;
        for (int k = 0; k < nds; ++k) {
            const knng_dataset& D = b->descs[g.members[k]];
            dsbase[k] = acc;
            acc += (uint32_t)D.N;
            st_init[k] = stream_state(D.seed, 1, 0);
            for (int t = 1; t <= T; ++t) st_table[(size_t)(t - 1) * nds + k] = stream_state(D.seed, 2, (uint64_t)t);
            oi[k] = D.d_ids;
            od[k] = D.d_dists;
            ix[k] = D.dX;
            idd[k] = D.d;
        }
        dsbase[nds] = acc;
        HIP_TRY(hipMemcpyAsync(tb + L.dsbase, dsbase.data(), dsbase.size() * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(tb + L.st_init, st_init.data(), st_init.size() * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(tb + L.st_table, st_table.data(), st_table.size() * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(tb + L.out_ids, oi.data(), oi.size() * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(tb + L.out_dists, od.data(), od.size() * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(tb + L.in_X, ix.data(), ix.size() * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(tb + L.in_d, idd.data(), idd.size() * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));   // host staging vectors go out of scope
    }
    return KNNG_OK;
}

// Enqueue one group's setup + init, or one iteration t, or its write-out.
void batch_group_setup(const BatchGroup& g, hipStream_t s) {
    const Views& v = g.v;
    launch_fill_u64(v.counters, 0ull, kNumCounters, s);
    launch_fill_u32(v.nn, 0u, v.N, s);
    launch_fill_u32(v.stop, 0u, 1, s);
    launch_batch_setup(v, s);
    if (g.path != KNNG_PATH_VALU) launch_norms(v, s);
    if (g.path == KNNG_PATH_MFMA_BF16X3) launch_make_split(v, s);
    launch_init(v, 0, g.path != KNNG_PATH_VALU ? kDistGram : kDistDirect, s);
}

void batch_group_iteration(const BatchGroup& g, int t, const knng_params& p, hipStream_t s) {
    const Views& v = g.v;
    // the hub list is per iteration (its count must not grow past N); the
    // other counters accumulate over the iterations (errors are read at the end)
    // once the group has stopped every pass below returns at entry
    launch_fill_u64(v.counters + kCntHubs, 0ull, 1, s, v.stop);
    launch_fill_u32(v.rdeg, 0u, 4 * (int64_t)v.N, s, v.stop);
    launch_fill_u32(v.chg, 0u, (int64_t)v.N, s, v.stop);
    if (v.rev_S) {
        launch_rev_partition(v, 0, t, s);
    } else {
        launch_rev_hist(v, s);
        launch_scan(v.rdeg, v.roff, v.N, v.scan_tmp, s, v.stop);
        launch_rev_scatter(v, 0, t, s);
    }
    launch_select(v, 0, t, s);
    launch_scan(v.cap, v.poff, v.N, v.scan_tmp, s, v.stop);
    if (g.path == KNNG_PATH_MFMA_BF16X3)
        launch_join_split(v, s);
    else if (g.path == KNNG_PATH_MFMA)
        launch_join_mfma(v, s);
    else
        launch_join_valu(v, s);
    launch_merge(v, s);
    launch_scan(v.chg, v.chgoff, v.N, v.scan_tmp, s, v.stop);
    launch_batch_step(v, t, p.max_iters, p.K, p.delta, s);
}

void batch_enqueue(knng_batch* b, hipStream_t s) {
    // larger groups first: they set the critical path
    for (const auto& g : b->groups) batch_group_setup(g, s);
    for (int t = 1; t <= b->p.max_iters; ++t)
        for (const auto& g : b->groups) batch_group_iteration(g, t, b->p, s);
    for (const auto& g : b->groups) launch_batch_finalize(g.v, s);
}

// Autotuner: for every d, each candidate (join path, workgroup cap of the
// select and join passes) runs the whole build of that dimension's datasets
// (setup untimed; every iteration up to T, a stopped group's passes return at
// entry) timed with HIP events, and the fastest is kept. Paths: the direct
// form always, the matrix forms where 2C <= 64. Caps: one workgroup per four
// owners (at most 65536), or eight workgroups per compute unit looping over
// the owners, which costs less once most datasets have converged.
knng_status batch_autotune(knng_batch* b, hipStream_t s) {
    std::string table;
    std::vector<int> ds_seen;
    for (const auto& D : b->descs)
        if (std::find(ds_seen.begin(), ds_seen.end(), D.d) == ds_seen.end()) ds_seen.push_back(D.d);
    std::sort(ds_seen.begin(), ds_seen.end());
    const int C = sample_cap(b->p.K, b->p.rho);
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int caps[2] = {0, 8 * std::max(cus, 1)};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    for (int d : ds_seen) {
        int best_path = d >= kAutoMatrixMinD && 2 * C <= 64 ? KNNG_PATH_MFMA_BF16X3 : KNNG_PATH_VALU, best_cap = 0;
        float best_ms = 1e30f;
        for (int path : {KNNG_PATH_VALU, KNNG_PATH_MFMA, KNNG_PATH_MFMA_BF16X3}) {
            if (path != KNNG_PATH_VALU && 2 * C > 64) continue;
            for (int cap : caps) {
                knng_batch tb;
                tb.p = b->p;
                tb.p.path = path;
                for (const auto& D : b->descs)
                    if (D.d == d) tb.descs.push_back(D);
                size_t total = 0;
                if (batch_groups(tb.descs.data(), (int32_t)tb.descs.size(), &tb.p, "", tb.groups, total) != KNNG_OK)
                    continue;
                if (total > b->ws_bytes) continue;
                for (auto& g : tb.groups) g.cap = cap;
                tb.ws = b->ws;
                tb.ws_bytes = b->ws_bytes;
                if (batch_upload(&tb, s) != KNNG_OK) continue;
                for (const auto& g : tb.groups) batch_group_setup(g, s);
                HIP_TRY(hipEventRecord(e0, s));
                for (int t = 1; t <= tb.p.max_iters; ++t)
                    for (const auto& g : tb.groups) batch_group_iteration(g, t, tb.p, s);
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipStreamSynchronize(s));
                const float ms = ms_between(e0, e1);
                if (ms >= 0.f && ms < best_ms) {
                    best_ms = ms;
                    best_path = path;
                    best_cap = cap;
                }
            }
        }
        if (!table.empty()) table += ",";
        table += tuned_entry(d, best_path, best_cap);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tuning = table;
    return KNNG_OK;
}

}  // namespace

extern "C" {

size_t knng_batch_workspace_bytes(const knng_dataset* descs, int32_t n, const knng_params* params) {
    if (batch_validate(descs, n, params) != KNNG_OK) return 0;
    // room for any join path of every group (the autotuner may pick any): the
    // split form needs the most of each group, so its uniform layout bounds a mix
    size_t best = 0;
    for (int path : {KNNG_PATH_VALU, KNNG_PATH_MFMA, KNNG_PATH_MFMA_BF16X3}) {
        knng_params p = *params;
        if (params->path != KNNG_PATH_AUTO && params->path != path) continue;
        p.path = path;
        std::vector<BatchGroup> groups;
        size_t total = 0;
        if (batch_groups(descs, n, &p, "", groups, total) == KNNG_OK) best = std::max(best, total);
    }
    knng_params p = *params;
    std::vector<BatchGroup> groups;
    size_t total = 0;
    if (batch_groups(descs, n, &p, "", groups, total) == KNNG_OK) best = std::max(best, total);
    if (best == 0) (void)fail(KNNG_EINVAL, "no valid layout for these datasets");
    return best;
}

knng_status knng_batch_plan(knng_batch** out, const knng_dataset* descs, int32_t n, const knng_params* params,
                            void* d_ws, size_t ws_bytes, const char* tuning, void* stream) {
    g_err.clear();
    if (!out) return fail(KNNG_EINVAL, "out is NULL");
    *out = nullptr;
    knng_status s = batch_validate(descs, n, params);
    if (s != KNNG_OK) return s;
    if (!d_ws) return fail(KNNG_EINVAL, "workspace is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    knng_batch* b = new (std::nothrow) knng_batch();
    if (!b) return fail(KNNG_ENOMEM, "host allocation of the plan failed");
    b->p = *params;
    b->descs.assign(descs, descs + n);
    b->ws = static_cast<char*>(d_ws);
    b->ws_bytes = ws_bytes;
    if (params->path == KNNG_PATH_AUTO && (!tuning || !*tuning || std::string(tuning) == "auto")) {
        s = batch_autotune(b, st);
        if (s != KNNG_OK) {
            delete b;
            return s;
        }
    } else {
        b->tuning = tuning ? tuning : "";
    }
    size_t total = 0;
    s = batch_groups(descs, n, params, b->tuning, b->groups, total);
    if (s != KNNG_OK) {
        delete b;
        return s;
    }
    if (total > ws_bytes) {
        delete b;
        char buf[128];
        snprintf(buf, sizeof buf, "workspace too small: %zu < %zu bytes", ws_bytes, total);
        return fail(KNNG_ENOMEM, buf);
    }
    std::sort(b->groups.begin(), b->groups.end(), [](const BatchGroup& x, const BatchGroup& y) {
        return (double)x.N * x.dp > (double)y.N * y.dp;
    });
    s = batch_upload(b, st);
    if (s != KNNG_OK) {
        delete b;
        return s;
    }
    // finiteness of every input (once, here, so that execute needs no read-back)
    uint64_t hc[kNumCounters];
    for (const auto& g : b->groups) {
        launch_fill_u64(g.v.counters, 0ull, kNumCounters, st);
        launch_batch_setup(g.v, st);
        if (hipMemcpyAsync(hc, g.v.counters, sizeof hc, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            delete b;
            return fail(KNNG_EDEVICE, "batch setup failed");
        }
        if (hc[kCntNonFinite]) {
            delete b;
            return fail(KNNG_EINVAL, "a dataset holds a NaN or an infinity");
        }
    }
    *out = b;
    return KNNG_OK;
}

const char* knng_batch_tuning(const knng_batch* b) { return b ? b->tuning.c_str() : ""; }

knng_status knng_batch_execute(knng_batch* b, void* stream) {
    if (!b) return fail(KNNG_EINVAL, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    batch_enqueue(b, s);
    HIP_TRY(hipGetLastError());
    return KNNG_OK;
}

knng_status knng_batch_capture(knng_batch* b, void* stream) {
    if (!b) return fail(KNNG_EINVAL, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!s) return fail(KNNG_EINVAL, "capture needs a non-default stream");
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    batch_enqueue(b, s);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(s, &g));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return KNNG_OK;
}

knng_status knng_batch_launch(knng_batch* b, void* stream) {
    if (!b || !b->exec) return fail(KNNG_EINVAL, "no captured graph: call knng_batch_capture first");
    HIP_TRY(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
    return KNNG_OK;
}

knng_status knng_batch_stats(knng_batch* b, int32_t* iters, int32_t* converged, int64_t* evals, int64_t* changes,
                             void* stream) {
    if (!b) return fail(KNNG_EINVAL, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int T = b->p.max_iters;
    for (const auto& g : b->groups) {
        const int nds = (int)g.members.size();
        std::vector<int32_t> it(nds), cv(nds);
        std::vector<int64_t> st((size_t)nds * T * 2);
        uint64_t hc[kNumCounters];
        HIP_TRY(hipMemcpyAsync(it.data(), g.v.ds_iters, nds * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(cv.data(), g.v.ds_conv, nds * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(st.data(), g.v.ds_stats, st.size() * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hc, g.v.counters, sizeof hc, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hc[kCntError]) {
            char buf[96];
            snprintf(buf, sizeof buf, "device invariant failed in a batched build (code %llu)",
                     (unsigned long long)hc[kCntError]);
            return fail(KNNG_EDEVICE, buf);
        }
        for (int k = 0; k < nds; ++k) {
            const int i = g.members[k];
            if (iters) iters[i] = it[k];
            if (converged) converged[i] = cv[k];
            for (int t = 0; t < T; ++t) {
                const bool run = t < it[k];
                if (evals) evals[(size_t)i * T + t] = run ? st[((size_t)k * T + t) * 2] : 0;
                if (changes) changes[(size_t)i * T + t] = run ? st[((size_t)k * T + t) * 2 + 1] : 0;
            }
        }
    }
    return KNNG_OK;
}

void knng_batch_destroy(knng_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
}

}  // extern "C"
