// Host orchestrator and C ABI (include/knng.h) of the gfx950 NN-Descent library.
//
// One build: pad rows -> random initial graph (Sec. 2) -> iterations of
// {reverse bucketing + weighted sampling (Sec. 3.1), local join (Sec. 2,
// Sec. 3.3), top-K merge} until changes < delta*N*K (Sec. 2) -> optional
// graph-ordered permutation after iteration 1 (Sec. 3.2) -> write-out in
// original order. All device memory comes from the caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <utility>
#include <cstring>
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
    int C;
    int64_t pmax;    // proposal slots
    size_t total;
    // byte offsets
    size_t o_Xp, o_nrm, o_orig, o_posof, o_lkey, o_lpos, o_cnt4, o_roff, o_rev, o_cand, o_nn, o_big, o_hubs, o_poff,
        o_pkey, o_ppos, o_scan, o_counters, o_partial, o_Xb, o_nb, o_Xb2, o_nb2, o_comp, o_comp2, o_par, o_lvl, o_best, o_size, o_offs,
        o_cur, o_newpos, o_lkey2, o_lpos2, o_Xp2, o_nrm2, o_orig2, o_flag;
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
    if (p->path < KNNG_PATH_AUTO || p->path > KNNG_PATH_MFMA) return fail(KNNG_EINVAL, "unknown path");
    if (N * (int64_t)p->K >= (1LL << 31)) return fail(KNNG_EINVAL, "N*K must be < 2^31");
    return KNNG_OK;
}

knng_status make_plan(int64_t N, int32_t d, const knng_params* p, Plan& P) {
    knng_status s = validate(N, d, p);
    if (s != KNNG_OK) return s;
    const int K = p->K;
    P.C = sample_cap(K, p->rho);
    int path = p->path;
    P.bf16 = p->precision == KNNG_BF16_SCREEN ? 1 : 0;
    if (P.bf16) {
        if (path == KNNG_PATH_VALU) return fail(KNNG_EINVAL, "the BF16-screened form runs on the MFMA path");
        path = KNNG_PATH_MFMA;
    }
    if (path == KNNG_PATH_AUTO) path = (d >= 64 && 2 * P.C <= 64) ? KNNG_PATH_MFMA : KNNG_PATH_VALU;
    if (path == KNNG_PATH_MFMA && 2 * P.C > 64) return fail(KNNG_EINVAL, "MFMA path needs ceil(rho*K) <= 32");
    P.path = path;
    P.reorder = p->reorder ? 1 : 0;
    P.dp = (int)(path == KNNG_PATH_MFMA ? round_up(d, 32) : round_up(d, 4));
    if (path == KNNG_PATH_VALU) {
        Views tv{};
        tv.C = P.C;
        tv.dp = P.dp;
        if (!join_valu_fits(tv))
            return fail(KNNG_EINVAL, "VALU path: 2*C rows of d floats do not fit the LDS stage; use the MFMA path");
    }
    const int64_t C = P.C;
    const int64_t per_node = C * (C - 1) + 2 * C * C;  // 2 e(u) at most
    P.pmax = N * per_node;
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
    P.o_orig = take((size_t)N * 4);
    P.o_posof = take((size_t)N * 4);
    P.o_lkey = take(NK * 8);
    P.o_lpos = take(NK * 4);
    P.o_cnt4 = take((size_t)N * 4 * 4);   // rdeg, rcur, cap, pcnt: one fill
    P.o_roff = take(((size_t)N + 1) * 4);
    P.o_rev = take(NK * 16);
    P.o_cand = take((size_t)N * 2 * C * 8);
    P.o_nn = take((size_t)N * 4);
    P.o_big = take((size_t)N * 4);
    P.o_hubs = take((size_t)N * 4);
    P.o_poff = take(((size_t)N + 1) * 4);
    P.o_pkey = take((size_t)P.pmax * 8);
    P.o_ppos = take((size_t)P.pmax * 4);
    P.o_scan = take(scan_tmp_words((int)N) * 4);
    P.o_counters = take(kNumCounters * 8);
    P.o_partial = take(partial_words() * 8);
    if (P.bf16) {
        P.o_Xb = take((size_t)N * P.dp * 2);
        P.o_nb = take((size_t)N * 4);
        if (p->reorder) {
            P.o_Xb2 = take((size_t)N * P.dp * 2);
            P.o_nb2 = take((size_t)N * 4);
        }
    }
    if (p->reorder) {   // permutation scratch only when the permutation is on
        P.o_comp = take((size_t)N * 4);
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
        P.o_Xp2 = take((size_t)N * P.dp * 4);
        P.o_nrm2 = take((size_t)N * 4);
        P.o_orig2 = take((size_t)N * 4);
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
    v.Xp = reinterpret_cast<float*>(b + P.o_Xp);
    v.nrm = reinterpret_cast<float*>(b + P.o_nrm);
    v.orig = reinterpret_cast<int32_t*>(b + P.o_orig);
    v.posof = reinterpret_cast<int32_t*>(b + P.o_posof);
    v.lkey = reinterpret_cast<uint64_t*>(b + P.o_lkey);
    v.lpos = reinterpret_cast<uint32_t*>(b + P.o_lpos);
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
    v.ppos = reinterpret_cast<uint32_t*>(b + P.o_ppos);
    v.scan_tmp = reinterpret_cast<uint32_t*>(b + P.o_scan);
    v.counters = reinterpret_cast<uint64_t*>(b + P.o_counters);
    v.partial = reinterpret_cast<uint64_t*>(b + P.o_partial);
    if (P.bf16) {
        v.Xb = reinterpret_cast<uint16_t*>(b + P.o_Xb);
        v.nb = reinterpret_cast<float*>(b + P.o_nb);
        if (P.reorder) {
            v.Xb2 = reinterpret_cast<uint16_t*>(b + P.o_Xb2);
            v.nb2 = reinterpret_cast<float*>(b + P.o_nb2);
        }
    }
    if (P.reorder) {
        v.comp = reinterpret_cast<int32_t*>(b + P.o_comp);
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
        v.Xp2 = reinterpret_cast<float*>(b + P.o_Xp2);
        v.nrm2 = reinterpret_cast<float*>(b + P.o_nrm2);
        v.orig2 = reinterpret_cast<int32_t*>(b + P.o_orig2);
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

struct knng_ctx {
    Views v;
    Plan plan;
    knng_params p;
    int64_t N;
    int32_t d;
    hipStream_t stream;
    const float* dX;
    int t;               // iterations completed
    bool permuted;
    int perm_levels;
    bool has_graph;
    knng_stats stats;
    hipEvent_t ev[6];
    uint64_t hc[kNumCounters];
};

namespace {

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
    HIP_TRY(hipEventRecord(c->ev[4], s));
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
    std::swap(v.orig, v.orig2);
    std::swap(v.lkey, v.lkey2);
    std::swap(v.lpos, v.lpos2);
    std::swap(v.Xb, v.Xb2);
    std::swap(v.nb, v.nb2);
    launch_perm_posof(v, s);
    HIP_TRY(hipEventRecord(c->ev[5], s));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    c->stats.reorder_ms = ms_between(c->ev[4], c->ev[5]);
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

knng_status do_iterate(knng_ctx* c, int64_t* evals, int64_t* changes) {
    if (!c->has_graph) return fail(KNNG_EINVAL, "no graph: call knng_init_graph or knng_load_graph first");
    if (c->t >= KNNG_MAX_ITERS) return fail(KNNG_EINVAL, "iteration limit of the statistics reached");
    const Views& v = c->v;
    hipStream_t s = c->stream;
    const int t = c->t + 1;
    const uint64_t st = stream_state(c->p.seed, 2, (uint64_t)t);
    launch_fill_u32(v.rdeg, 0u, 4 * (int64_t)v.N, s);
    launch_fill_u64(v.counters, 0ull, kNumCounters, s);
    HIP_TRY(hipEventRecord(c->ev[0], s));
    launch_rev_hist(v, s);
    launch_scan(v.rdeg, v.roff, v.N, v.scan_tmp, s);
    launch_rev_scatter(v, st, s);
    launch_select(v, st, s);
    launch_scan(v.cap, v.poff, v.N, v.scan_tmp, s);
    HIP_TRY(hipEventRecord(c->ev[1], s));
    if (c->plan.bf16)
        launch_join_bf16(v, s);
    else if (c->plan.path == KNNG_PATH_MFMA)
        launch_join_mfma(v, s);
    else
        launch_join_valu(v, s);
    HIP_TRY(hipEventRecord(c->ev[2], s));
    launch_merge(v, s);
    launch_finish_counters(v, s);
    HIP_TRY(hipEventRecord(c->ev[3], s));
    HIP_TRY(hipGetLastError());
    knng_status st2 = read_counters(c);
    if (st2 != KNNG_OK) return st2;
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
    S.sample_ms[i] = ms_between(c->ev[0], c->ev[1]);
    S.join_ms[i] = ms_between(c->ev[1], c->ev[2]);
    S.merge_ms[i] = ms_between(c->ev[2], c->ev[3]);
    S.iter_ms[i] = ms_between(c->ev[0], c->ev[3]);
    S.iters = t;
    c->t = t;
    if (t == 1 && c->p.reorder && !c->permuted) {
        knng_status ps = do_permute(c);
        if (ps != KNNG_OK) return ps;
    }
    if (evals) *evals = e;
    if (changes) *changes = ch;
    return KNNG_OK;
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
    c->plan = P;
    c->p = *params;
    c->N = N;
    c->d = d;
    c->stream = static_cast<hipStream_t>(stream);
    c->dX = dX;
    c->v = carve(P, N, d, params->K, d_ws);
    std::memset(&c->stats, 0, sizeof(c->stats));
    c->stats.path = P.path;
    c->stats.precision = P.bf16 ? KNNG_BF16_SCREEN : KNNG_FP32;
    c->stats.dpad = P.dp;
    for (auto& e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            knng_destroy(c);
            return fail(KNNG_EDEVICE, "hipEventCreate failed");
        }
    }
    launch_fill_u64(c->v.counters, 0ull, kNumCounters, c->stream);
    launch_pad_rows(dX, c->v, c->stream);
    if (P.path == KNNG_PATH_MFMA) launch_norms(c->v, c->stream);
    if (P.bf16) launch_make_bf16(c->v, c->stream);
    if (hipGetLastError() != hipSuccess || read_counters(c) != KNNG_OK) {
        knng_destroy(c);
        return fail(KNNG_EDEVICE, "row padding failed");
    }
    if (c->hc[kCntNonFinite]) {
        knng_destroy(c);
        return fail(KNNG_EINVAL, "X holds a NaN or an infinity");
    }
    *out = c;
    return KNNG_OK;
}

knng_status knng_init_graph(knng_ctx* c) {
    if (!c) return fail(KNNG_EINVAL, "ctx is NULL");
    if (c->permuted) return fail(KNNG_EINVAL, "init after permutation is not supported");
    launch_init(c->v, stream_state(c->p.seed, 1, 0), c->plan.path == KNNG_PATH_MFMA && !c->plan.bf16, c->stream);
    HIP_TRY(hipGetLastError());
    c->t = 0;
    c->has_graph = true;
    return KNNG_OK;
}

knng_status knng_load_graph(knng_ctx* c, const int32_t* d_ids, const uint8_t* d_flags, int32_t t) {
    if (!c) return fail(KNNG_EINVAL, "ctx is NULL");
    if (!d_ids || !d_flags) return fail(KNNG_EINVAL, "ids/flags are NULL");
    if (c->permuted) return fail(KNNG_EINVAL, "load after permutation is not supported");
    if (t < 0 || t >= KNNG_MAX_ITERS) return fail(KNNG_EINVAL, "t out of range");
    launch_fill_u64(c->v.counters, 0ull, kNumCounters, c->stream);
    launch_load_rows(c->v, d_ids, d_flags, c->plan.path == KNNG_PATH_MFMA && !c->plan.bf16, c->stream);
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
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

knng_status knng_build(const float* dX, int64_t N, int32_t d, const knng_params* params, int32_t* d_ids,
                       float* d_dists, void* d_ws, size_t ws_bytes, void* stream, knng_stats* stats) {
    if (!d_ids || !d_dists) return fail(KNNG_EINVAL, "outputs are NULL");
    knng_ctx* c = nullptr;
    knng_status s = knng_create(&c, dX, N, d, params, d_ws, ws_bytes, stream);
    if (s != KNNG_OK) return s;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess || hipEventCreate(&e2) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        knng_destroy(c);
        return fail(KNNG_EDEVICE, "hipEventCreate failed");
    }
    auto cleanup = [&]() {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
        knng_destroy(c);
    };
    (void)hipEventRecord(e0, c->stream);
    s = knng_init_graph(c);
    if (s != KNNG_OK) { cleanup(); return s; }
    (void)hipEventRecord(e1, c->stream);
    const double thr = (double)params->delta * (double)N * (double)params->K;
    bool conv = false;
    for (int it = 0; it < params->max_iters; ++it) {
        int64_t e = 0, ch = 0;
        s = do_iterate(c, &e, &ch);
        if (s != KNNG_OK) { cleanup(); return s; }
        if ((double)ch < thr) { conv = true; break; }
    }
    launch_finalize(c->v, d_ids, d_dists, nullptr, c->stream);
    (void)hipEventRecord(e2, c->stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        cleanup();
        return fail(KNNG_EDEVICE, "finalize failed");
    }
    c->stats.converged = conv ? 1 : 0;
    c->stats.init_ms = ms_between(e0, e1);
    c->stats.total_ms = ms_between(e0, e2);
    float fin = 0.f;
    if (hipEventElapsedTime(&fin, e0, e2) == hipSuccess) {
        float acc = c->stats.init_ms + c->stats.reorder_ms;
        for (int i = 0; i < c->stats.iters; ++i) acc += c->stats.iter_ms[i];
        c->stats.finalize_ms = fin - acc > 0.f ? fin - acc : 0.f;
    }
    if (stats) *stats = c->stats;
    cleanup();
    return (conv || params->max_iters == 0) ? KNNG_OK : KNNG_ENOTCONV;
}

}  // extern "C"
