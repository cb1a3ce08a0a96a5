// Device kernels of the NN-Descent iteration for gfx950 (CDNA4, wave64).
//
// Method: Kluser et al., "Fast single-core K-Nearest Neighbor Graph
// computation", arXiv 2112.06630.
//   init              Sec. 2 (random initial K-NNG)
//   reverse + select  Sec. 3.1 (neighbourhood = forward + reverse lists,
//                     fused weighted sampling of rho*k members)
//   join              Sec. 2 calculation step, Sec. 3.3 (squared l2, blocked
//                     pairwise distances within a neighbourhood)
//   merge             Sec. 2 / Fig. 1 (replace an edge when a closer vertex is found)
//   permutation       Sec. 3.2 (graph-driven memory reordering)
//
// Determinism: every weight is a hash of (seed, t, pair of original ids),
// every list is ordered by the 64-bit key (f32 bits of D << 32 | original id),
// and every selection is by rank over such keys, so no result depends on
// atomic or scheduling order.
#include "knng_impl.h"

namespace knng {

// ------------------------------------------------------------------ helpers

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Sampling weight of the unordered pair {a, b} (original ids); `st` is the
// per-(seed, tag, t) stream state prepared on the host.
__device__ __forceinline__ uint32_t pair_weight(uint64_t st, uint32_t a, uint32_t b) {
    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    return (uint32_t)(mix64(st ^ (((uint64_t)lo << 32) | hi)) >> 32);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t rl32(uint32_t x, int j) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, j);
}

__device__ __forceinline__ uint64_t rl64(uint64_t x, int j) {
    return ((uint64_t)rl32((uint32_t)(x >> 32), j) << 32) | rl32((uint32_t)x, j);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Cross-lane shuffles read the source lane's register only if that lane takes
// part: every shuffle below is evaluated by the whole wave, never inside a
// short-circuited condition.

// Orders the LDS traffic of one wavefront: LDS operations of a wave execute
// in issue order, so only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t x, int d) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}

// One compare-exchange step of a bitonic network across the wave: lanes
// lane and lane^j exchange; an ascending block keeps the smaller key in its
// lower lane. Equal keys are left in place.
__device__ __forceinline__ void cmpx(uint64_t& k, uint32_t& v, int j, bool asc) {
    const int lane = lane_id();
    const uint64_t ok = shfl_xor64(k, j);
    const uint32_t ov = (uint32_t)__shfl_xor((int)v, j);
    const bool low = (lane & j) == 0;
    const bool sw = (asc == low) ? (ok < k) : (ok > k);
    if (sw) {
        k = ok;
        v = ov;
    }
}

// Ascending bitonic sort of 64 (key, value) pairs, one per lane.
__device__ __forceinline__ void wave_sort(uint64_t& k, uint32_t& v) {
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) cmpx(k, v, j, (lane & size) == 0);
    }
}

// Sorts a bitonic sequence of 64 pairs ascending.
__device__ __forceinline__ void wave_bitonic_clean(uint64_t& k, uint32_t& v) {
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) cmpx(k, v, j, true);
}

__device__ __forceinline__ uint64_t key_of(float D, uint32_t id) {
    return ((uint64_t)__float_as_uint(D) << 32) | id;
}

// Squared l2 of two rows of dp floats (dp % 4 == 0), direct form. Four
// partial sums over j mod 4, combined as (s0+s1)+(s2+s3): one fixed order,
// and symmetric in (a, b) bit for bit since (x-y)^2 == (y-x)^2.
__device__ __forceinline__ float dist_direct(const float* __restrict__ a, const float* __restrict__ b, int dp) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int j = 0; j < dp; j += 4) {
        const float4 x = *reinterpret_cast<const float4*>(a + j);
        const float4 y = *reinterpret_cast<const float4*>(b + j);
        const float t0 = x.x - y.x, t1 = x.y - y.y, t2 = x.z - y.z, t3 = x.w - y.w;
        s0 = fmaf(t0, t0, s0);
        s1 = fmaf(t1, t1, s1);
        s2 = fmaf(t2, t2, s2);
        s3 = fmaf(t3, t3, s3);
    }
    return (s0 + s1) + (s2 + s3);
}

// Gram form ||a||^2 + ||b||^2 - 2 a.b with the dot product in the same
// four-partial-sum order; clamped at +0.
__device__ __forceinline__ float dist_gram_valu(const float* __restrict__ a, const float* __restrict__ b,
                                                int dp, float na, float nb) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int j = 0; j < dp; j += 4) {
        const float4 x = *reinterpret_cast<const float4*>(a + j);
        const float4 y = *reinterpret_cast<const float4*>(b + j);
        s0 = fmaf(x.x, y.x, s0);
        s1 = fmaf(x.y, y.y, s1);
        s2 = fmaf(x.z, y.z, s2);
        s3 = fmaf(x.w, y.w, s3);
    }
    const float dot = (s0 + s1) + (s2 + s3);
    const float D = (na + nb) - 2.0f * dot;
    return D > 0.f ? D : 0.f;
}

__device__ __forceinline__ float sq_norm(const float* __restrict__ a, int dp) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int j = 0; j < dp; j += 4) {
        const float4 x = *reinterpret_cast<const float4*>(a + j);
        s0 = fmaf(x.x, x.x, s0);
        s1 = fmaf(x.y, x.y, s1);
        s2 = fmaf(x.z, x.z, s2);
        s3 = fmaf(x.w, x.w, s3);
    }
    return (s0 + s1) + (s2 + s3);
}

// q = a / b for 0 <= a < 2^31, 1 <= b, via a double reciprocal and one fix-up.
__device__ __forceinline__ uint32_t udiv(uint32_t a, uint32_t b, double rcp) {
    uint32_t q = (uint32_t)((double)a * rcp);
    if (q * b > a) --q;
    else if ((q + 1) * b <= a) ++q;
    return q;
}

static inline int grid_for(int64_t items, int per_block, int cap = 1 << 20) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ------------------------------------------------------------------ fills

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 1024, 4096)), dim3(256), 0, s, p, v, n);
}

void launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 1024, 4096)), dim3(256), 0, s, p, v, n);
}

// ------------------------------------------------------------------ layout (a0)

// Rows padded to dp floats (zeros), identity permutation, finiteness check.
__global__ void k_pad_rows(const float* __restrict__ X, int N, int d, int dp, float* __restrict__ Xp,
                           int32_t* __restrict__ orig, int32_t* __restrict__ posof, uint64_t* counters) {
    const int64_t total = (int64_t)N * dp;
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / dp;
        const int c = (int)(i - r * dp);
        const float x = c < d ? X[r * d + c] : 0.f;
        bad |= (__float_as_uint(x) & 0x7f800000u) == 0x7f800000u;
        Xp[i] = x;
        if (c == 0) {
            orig[r] = (int32_t)r;
            posof[r] = (int32_t)r;
        }
    }
    if (bad) atomicOr((unsigned long long*)&counters[kCntNonFinite], 1ull);
}

void launch_pad_rows(const float* X, const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_rows, dim3(grid_for((int64_t)v.N * v.dp, 1024, 8192)), dim3(256), 0, s, X, v.N, v.d,
                       v.dp, v.Xp, v.orig, v.posof, v.counters);
}

__global__ void k_norms(const float* __restrict__ Xp, int N, int dp, float* __restrict__ nrm) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < N; r += gridDim.x * blockDim.x)
        nrm[r] = sq_norm(Xp + (size_t)r * dp, dp);
}

void launch_norms(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_norms, dim3(grid_for(v.N, 256, 8192)), dim3(256), 0, s, v.Xp, v.N, v.dp, v.nrm);
}

// ------------------------------------------------------------------ init (a1)

constexpr int kRowWaves = 4;

// Lanes < K hold one entry each (position `pid` of the neighbour, NEW flag in
// pf). Computes D against row u, ranks the K keys and writes the sorted row.
__device__ __forceinline__ void finish_row(const Views& v, int u, uint32_t pid, uint32_t pf, int gram) {
    const int lane = lane_id();
    const int K = v.K;
    uint64_t key = ~0ull;
    if (lane < K) {
        const float* a = v.Xp + (size_t)u * v.dp;
        const float* b = v.Xp + (size_t)pid * v.dp;
        const float D = gram ? dist_gram_valu(a, b, v.dp, v.nrm[u], v.nrm[pid]) : dist_direct(a, b, v.dp);
        key = key_of(D, (uint32_t)v.orig[pid]);
    }
    int rank = 0;
    for (int j = 0; j < K; ++j) rank += (rl64(key, j) < key) ? 1 : 0;
    if (lane < K) {
        v.lkey[(size_t)u * K + rank] = key;
        v.lpos[(size_t)u * K + rank] = pid | pf;
    }
}

// K distinct ids != u from H(seed,1,0,u,j), j = 0,1,...: the first K distinct
// draws in draw order, as in the oracle. Positions equal original ids here.
__global__ __launch_bounds__(256) void k_init(Views v, uint64_t st, int gram) {
    __shared__ uint32_t s_sel[kRowWaves][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int N = v.N, K = v.K;
    for (int u = blockIdx.x * kRowWaves + w; u < N; u += gridDim.x * kRowWaves) {
        int have = 0;
        for (uint32_t base = 0; have < K; base += 64) {
            const uint32_t j = base + (uint32_t)lane;
            const uint64_t h = mix64(st ^ (((uint64_t)(uint32_t)u << 32) | j));
            uint32_t c = (uint32_t)(((h >> 32) * (uint64_t)(uint32_t)(N - 1)) >> 32);
            c += (c >= (uint32_t)u) ? 1u : 0u;
            bool novel = true;
            for (int i = 0; i < have; ++i) novel &= (s_sel[w][i] != c);
            for (int i = 0; i < 63; ++i) {
                const uint32_t ci = rl32(c, i);
                novel &= !(i < lane && ci == c);
            }
            const uint64_t m = ballot(novel);
            const uint32_t r = mbcnt(m);
            wave_sync();
            if (novel && have + (int)r < K) s_sel[w][have + r] = c;
            wave_sync();
            have = min(K, have + __popcll(m));
        }
        const uint32_t pid = lane < K ? s_sel[w][lane] : 0u;
        wave_sync();
        finish_row(v, u, pid, kNewBit, gram);
    }
}

void launch_init(const Views& v, uint64_t st_init, int gram, hipStream_t s) {
    hipLaunchKernelGGL(k_init, dim3(grid_for(v.N, kRowWaves, 65536)), dim3(256), 0, s, v, st_init, gram);
}

// Load a caller state: ids are original ids (positions equal ids before any
// permutation); distances recomputed, rows re-sorted by key.
__global__ __launch_bounds__(256) void k_load_rows(Views v, const int32_t* __restrict__ ids,
                                                   const uint8_t* __restrict__ flags, int gram) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    for (int u = blockIdx.x * kRowWaves + w; u < v.N; u += gridDim.x * kRowWaves) {
        uint32_t pid = 0, pf = 0;
        if (lane < v.K) {
            pid = (uint32_t)ids[(size_t)u * v.K + lane];
            pf = flags[(size_t)u * v.K + lane] ? kNewBit : 0u;
        }
        // a row must hold K distinct ids in [0, N), none equal to u
        bool bad = lane < v.K && (pid >= (uint32_t)v.N || pid == (uint32_t)u);
        for (int j = 0; j < v.K; ++j) {
            const uint32_t pj = rl32(pid, j);
            bad |= lane < v.K && j != lane && pj == pid;
        }
        if (ballot(bad)) {
            if (lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 4ull);
            continue;
        }
        finish_row(v, u, pid, pf, gram);
    }
}

void launch_load_rows(const Views& v, const int32_t* ids, const uint8_t* flags, int gram, hipStream_t s) {
    hipLaunchKernelGGL(k_load_rows, dim3(grid_for(v.N, kRowWaves, 65536)), dim3(256), 0, s, v, ids, flags, gram);
}

// ------------------------------------------------------------------ scan

constexpr int kScanBlock = 1024;  // items per block (256 threads x 4)

size_t scan_tmp_words(int n) { return (size_t)(n / kScanBlock + 2) + 64; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

__global__ __launch_bounds__(256) void k_scan_local(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                    int n, uint32_t* __restrict__ bsum) {
    __shared__ uint32_t s_w[4];
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)t * 4;
    uint32_t a[4];
    for (int i = 0; i < 4; ++i) a[i] = (base + i < n) ? in[base + i] : 0u;
    const uint32_t loc = a[0] + a[1] + a[2] + a[3];
    const uint32_t inc = wave_incl_scan(loc);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t woff = 0;
    for (int i = 0; i < w; ++i) woff += s_w[i];
    uint32_t run = woff + inc - loc;
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) out[base + i] = run;
        run += a[i];
    }
    if (t == 255) bsum[blockIdx.x] = woff + inc;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ bsum, int nb) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
    if (t == 0) s_carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const uint32_t x = (b0 + t < nb) ? bsum[b0 + t] : 0u;
        const uint32_t inc = wave_incl_scan(x);
        if (lane == 63) s_w[w] = inc;
        __syncthreads();
        uint32_t woff = 0;
        for (int i = 0; i < w; ++i) woff += s_w[i];
        const uint32_t carry = s_carry;
        if (b0 + t < nb) bsum[b0 + t] = carry + woff + inc - x;
        __syncthreads();
        if (t == 1023) s_carry = carry + woff + inc;
        __syncthreads();
    }
    if (t == 0) bsum[nb] = s_carry;
}

__global__ void k_scan_add(uint32_t* __restrict__ out, int n, const uint32_t* __restrict__ bsum, int nb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += bsum[i / kScanBlock];
    if (i == 0) out[n] = bsum[nb];
}

void launch_scan(const uint32_t* in, uint32_t* out, int n, uint32_t* tmp, hipStream_t s) {
    const int nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_local, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, in, out, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, nb > 0 ? nb : 1);
    hipLaunchKernelGGL(k_scan_add, dim3((n + 256) / 256), dim3(256), 0, s, out, n, tmp, nb > 0 ? nb : 1);
}

// ------------------------------------------------------------------ reverse lists (a2)

__global__ void k_rev_hist(const uint32_t* __restrict__ lpos, int64_t NK, uint32_t* __restrict__ rdeg) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < NK; e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&rdeg[lpos[e] & kPosMask], 1u);
}

void launch_rev_hist(const Views& v, hipStream_t s) {
    const int64_t NK = (int64_t)v.N * v.K;
    hipLaunchKernelGGL(k_rev_hist, dim3(grid_for(NK, 256, 1 << 16)), dim3(256), 0, s, v.lpos, NK, v.rdeg);
}

// Each edge u->v (flag f) becomes the reverse entry {w, orig u, pos u | f} of v.
__global__ void k_rev_scatter(Views v, uint64_t st) {
    const int64_t NK = (int64_t)v.N * v.K;
    const double rk = 1.0 / v.K;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < NK; e += (int64_t)gridDim.x * blockDim.x) {
        const int u = (int)udiv((uint32_t)e, (uint32_t)v.K, rk);
        const uint32_t pf = v.lpos[e];
        const uint32_t tp = pf & kPosMask;
        const uint32_t ov = (uint32_t)v.lkey[e];
        const uint32_t ou = (uint32_t)v.orig[u];
        const uint32_t w = pair_weight(st, ou, ov);
        const uint32_t slot = v.roff[tp] + atomicAdd(&v.rcur[tp], 1u);
        v.rev[slot] = make_uint4(w, ou, (uint32_t)u | (pf & kNewBit), 0u);
    }
}

void launch_rev_scatter(const Views& v, uint64_t st, hipStream_t s) {
    const int64_t NK = (int64_t)v.N * v.K;
    hipLaunchKernelGGL(k_rev_scatter, dim3(grid_for(NK, 256, 1 << 16)), dim3(256), 0, s, v, st);
}

// ------------------------------------------------------------------ select (a2)
//
// Pool of owner u: its K forward entries then its reverse bucket. The select
// key of an entry is (old flag << 63) | (w << 31) | member id: NEW before OLD,
// then weight, then id. Identical keys (the same member reached forward and
// reverse with the same flag) count once. N_new = C smallest NEW keys,
// N_old = C smallest OLD keys minus members already in N_new.

constexpr int kSelWaves = 4;

struct SelLds {
    uint64_t key[kSelWaves][kSelectStage];
    uint32_t pos[kSelWaves][kSelectStage];
    uint16_t rank[kSelWaves][kSelectStage];
    int16_t twin[kSelWaves][kSelectStage];
    uint8_t dup[kSelWaves][kSelectStage];
    uint16_t src[kSelWaves][kSelectStage];   // forward list index of staged forward entries
    uint32_t hist[kSelWaves][512];
    uint64_t oldmask[kSelWaves];
    uint32_t cnt[kSelWaves][2];
};

__device__ __forceinline__ void pool_entry(const Views& v, uint64_t st, int u, uint32_t ou, uint32_t rb, int i,
                                           uint64_t& key, uint32_t& pos, uint32_t& w) {
    uint32_t id, pf;
    if (i < v.K) {
        const size_t e = (size_t)u * v.K + i;
        id = (uint32_t)v.lkey[e];
        pf = v.lpos[e];
        w = pair_weight(st, ou, id);
    } else {
        const uint4 r = v.rev[rb + (uint32_t)(i - v.K)];
        w = r.x;
        id = r.y;
        pf = r.z;
    }
    pos = pf;
    key = ((uint64_t)((pf & kNewBit) ? 0u : 1u) << 63) | ((uint64_t)w << 31) | id;
}

// Radix prefilter for large pools: per flag, find a weight threshold T_f so
// that {w <= T_f} holds at least 2C entries of that flag (>= C distinct,
// since a member appears at most twice) and at most half the stage.
__device__ void select_radix_thresholds(const Views& v, uint64_t st, int u, uint32_t ou, uint32_t rb, int P,
                                        uint32_t* hist, uint32_t T[2]) {
    const int lane = lane_id();
    const uint32_t need = 2u * (uint32_t)v.C;
    uint32_t pref[2] = {0u, 0u}, below[2] = {0u, 0u};
    bool done[2] = {false, false};
    T[0] = T[1] = 0xffffffffu;
    for (int s = 24; s >= 0; s -= 8) {
        if (done[0] && done[1]) break;
        for (int i = lane; i < 512; i += 64) hist[i] = 0u;
        wave_sync();
        for (int i = lane; i < P; i += 64) {
            uint64_t key;
            uint32_t pos, w;
            pool_entry(v, st, u, ou, rb, i, key, pos, w);
            const int f = (int)(key >> 63);
            const bool match = (s == 24) || ((w >> (s + 8)) == (pref[f] >> (s + 8)));
            if (!done[f] && match) atomicAdd(&hist[f * 256 + ((w >> s) & 255u)], 1u);
        }
        wave_sync();
        for (int f = 0; f < 2; ++f) {
            if (done[f]) continue;
            uint32_t c[4];
            for (int q = 0; q < 4; ++q) c[q] = hist[f * 256 + lane * 4 + q];
            const uint32_t loc = c[0] + c[1] + c[2] + c[3];
            const uint32_t inc = wave_incl_scan(loc);
            const uint32_t exc = inc - loc;
            const uint32_t total = rl32(inc, 63);
            uint32_t b = 255u, cum_excl = below[f] + total, cum_incl = below[f] + total;
            // first lane whose inclusive count reaches `need`
            const uint64_t hit = ballot(below[f] + inc >= need);
            if (hit) {
                const int hl = __ffsll((long long)hit) - 1;
                uint32_t run = below[f] + rl32(exc, hl);
                uint32_t cc[4];
                for (int q = 0; q < 4; ++q) cc[q] = rl32(c[q], hl);
                for (int q = 0; q < 4; ++q) {
                    if (run + cc[q] >= need) {
                        b = (uint32_t)(hl * 4 + q);
                        cum_excl = run;
                        cum_incl = run + cc[q];
                        break;
                    }
                    run += cc[q];
                }
            }
            pref[f] |= b << s;
            below[f] = cum_excl;
            if (!hit || cum_incl <= (uint32_t)kSelectStage / 2 || s == 0) {
                done[f] = true;
                T[f] = hit ? (pref[f] | ((s > 0) ? ((1u << s) - 1u) : 0u)) : 0xffffffffu;
            }
        }
        wave_sync();
    }
}

// Pools of more than 64 entries (owners with a large reverse in-degree):
// staged in LDS (after a radix prefilter when they exceed the stage), ranks
// by counting over the stage.
__global__ __launch_bounds__(256) void k_select_large(Views v, uint64_t st) {
    __shared__ SelLds L;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int K = v.K, C = v.C;
    uint64_t* skey = L.key[w];
    uint32_t* spos = L.pos[w];
    const int nbig = (int)v.counters[kCntBig];
    for (int bi = blockIdx.x * kSelWaves + w; bi < nbig; bi += gridDim.x * kSelWaves) {
        const int u = (int)v.big[bi];
        const uint32_t rb = v.roff[u];
        const int P = K + (int)(v.roff[u + 1] - rb);
        const uint32_t ou = (uint32_t)v.orig[u];
        // ---- stage the pool (forward entries first) ----
        int n = 0, nf = 0;
        if (P <= kSelectStage) {
            for (int i = lane; i < P; i += 64) {
                uint64_t key;
                uint32_t pos, wt;
                pool_entry(v, st, u, ou, rb, i, key, pos, wt);
                skey[i] = key;
                spos[i] = pos;
                L.src[w][i] = (uint16_t)i;
            }
            n = P;
            nf = K;
        } else {
            uint32_t T[2];
            select_radix_thresholds(v, st, u, ou, rb, P, L.hist[w], T);
            for (int i0 = 0; i0 < P; i0 += 64) {
                const int i = i0 + lane;
                uint64_t key = 0;
                uint32_t pos = 0, wt = 0;
                bool keep = false;
                if (i < P) {
                    pool_entry(v, st, u, ou, rb, i, key, pos, wt);
                    keep = wt <= T[key >> 63];
                }
                const uint64_t m = ballot(keep);
                const int slot = n + (int)mbcnt(m);
                if (keep && slot < kSelectStage) {
                    skey[slot] = key;
                    spos[slot] = pos;
                    L.src[w][slot] = (uint16_t)(i < K ? i : 0);
                }
                n += __popcll(m);
                if (i0 < K) nf += __popcll(ballot(keep && i < K));
            }
            if (n > kSelectStage) {
                if (lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 1ull);
                n = kSelectStage;
            }
        }
        wave_sync();
        // ---- duplicates: a staged reverse entry equal to a staged forward entry ----
        for (int i = lane; i < n; i += 64) {
            bool dup = false;
            if (i >= nf) {
                const uint64_t ki = skey[i];
                for (int j = 0; j < nf; ++j) dup |= (skey[j] == ki);
            }
            L.dup[w][i] = dup ? 1 : 0;
        }
        wave_sync();
        // ---- ranks among distinct keys; twin = NEW entry of the same member ----
        uint32_t nvnew = 0, nvold = 0;
        for (int i0 = 0; i0 < n; i0 += 64) {
            const int i = i0 + lane;
            const bool valid = i < n && !L.dup[w][i];
            const uint64_t ki = i < n ? skey[i] : ~0ull;
            nvnew += __popcll(ballot(valid && !(ki >> 63)));
            nvold += __popcll(ballot(valid && (ki >> 63)));
        }
        for (int i0 = 0; i0 < n; i0 += 64) {
            const int i = i0 + lane;
            const uint64_t ki = i < n ? skey[i] : ~0ull;
            const uint64_t tk = ki & ~(1ull << 63);
            const bool is_old = (ki >> 63) != 0;
            uint32_t rank = 0;
            int twin = -1;
            for (int j = 0; j < n; ++j) {
                const uint64_t kj = skey[j];
                if (!L.dup[w][j]) {
                    rank += (kj < ki) ? 1u : 0u;
                    if (is_old && kj == tk) twin = j;
                }
            }
            if (i < n) {
                L.rank[w][i] = (uint16_t)rank;
                L.twin[w][i] = (int16_t)twin;
            }
        }
        if (lane == 0) L.oldmask[w] = 0ull;
        wave_sync();
        const uint32_t nnew = min((uint32_t)C, nvnew);
        // ---- old entries whose member is sampled as new are removed ----
        for (int i = lane; i < n; i += 64) {
            if (L.dup[w][i] || !(skey[i] >> 63)) continue;
            const uint32_t ro = L.rank[w][i] - nvnew;
            if (ro >= (uint32_t)C) continue;
            const int tw = L.twin[w][i];
            if (tw >= 0 && L.rank[w][tw] < (uint32_t)C)
                atomicOr((unsigned long long*)&L.oldmask[w], 1ull << ro);
        }
        wave_sync();
        const uint64_t omask = L.oldmask[w];
        const uint32_t nold = min((uint32_t)C, nvold) - (uint32_t)__popcll(omask);
        // ---- outputs: sampled sets, flips, per-target proposal capacities ----
        uint2* cs = v.cand + (size_t)u * 2 * C;
        for (int i = lane; i < n; i += 64) {
            if (L.dup[w][i]) continue;
            const uint64_t ki = skey[i];
            const uint32_t pf = spos[i];
            const uint32_t pos = pf & kPosMask;
            const uint32_t id = (uint32_t)(ki & 0x7fffffffu);
            const uint32_t rank = L.rank[w][i];
            if (!(ki >> 63)) {
                if (rank < (uint32_t)C) {
                    cs[rank] = make_uint2(id, pos);
                    if (nnew > 0) atomicAdd(&v.cap[pos], nnew - 1 + nold);
                    if (i < nf) v.lpos[(size_t)u * K + L.src[w][i]] = pos;  // flip NEW -> OLD
                }
            } else {
                const uint32_t ro = rank - nvnew;
                if (ro < (uint32_t)C && !((omask >> ro) & 1ull)) {
                    const uint32_t slot = nnew + ro - (uint32_t)__popcll(omask & ((1ull << ro) - 1ull));
                    cs[slot] = make_uint2(id, pos);
                    if (nnew > 0) atomicAdd(&v.cap[pos], nnew);
                }
            }
        }
        if (lane == 0) v.nn[u] = nnew | (nold << 16);
        wave_sync();
    }
}

// Pools of at most 64 entries, one per lane, in registers. Select key
// (w << 32) | (id << 1) | old: sorting it puts the two copies of a member
// reached by both routes with the same flag next to each other (the second
// is a duplicate), and a member's NEW entry right before its OLD entry.
// Ranks per flag are ballot prefix counts over the sorted lanes.
__global__ __launch_bounds__(256) void k_select_small(Views v, uint64_t st) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int N = v.N, K = v.K;
    const uint32_t C = (uint32_t)v.C;
    for (int u = blockIdx.x * kSelWaves + w; u < N; u += gridDim.x * kSelWaves) {
        const uint32_t rb = v.roff[u];
        const int P = K + (int)(v.roff[u + 1] - rb);
        if (P > 64) {
            if (lane == 0) {
                const uint32_t slot = (uint32_t)atomicAdd((unsigned long long*)&v.counters[kCntBig], 1ull);
                v.big[slot] = (uint32_t)u;
            }
            continue;
        }
        const uint32_t ou = (uint32_t)v.orig[u];
        uint64_t key = ~0ull;
        uint32_t pos = 0;
        if (lane < P) {
            uint32_t id, pf, wt;
            if (lane < K) {
                const size_t e = (size_t)u * K + lane;
                id = (uint32_t)v.lkey[e];
                pf = v.lpos[e];
                wt = pair_weight(st, ou, id);
            } else {
                const uint4 r = v.rev[rb + (uint32_t)(lane - K)];
                wt = r.x;
                id = r.y;
                pf = r.z;
            }
            key = ((uint64_t)wt << 32) | ((uint64_t)id << 1) | ((pf & kNewBit) ? 0u : 1u);
            pos = pf & kPosMask;
        }
        uint32_t idx = (uint32_t)lane;
        wave_sort(key, idx);
        const uint32_t mpos = (uint32_t)__shfl((int)pos, (int)idx);
        const uint64_t p1 = shfl_up64(key, 1), p2 = shfl_up64(key, 2);
        const bool real = key != ~0ull;
        const bool dup = real && lane >= 1 && p1 == key;
        const bool valid = real && !dup;
        const bool isnew = (key & 1ull) == 0;
        const uint64_t mnew = ballot(valid && isnew), mold = ballot(valid && !isnew);
        const uint32_t rnew = mbcnt(mnew), rold = mbcnt(mold);
        const bool seln = valid && isnew && rnew < C;
        const bool s1 = __shfl_up(seln ? 1 : 0, 1) != 0, s2 = __shfl_up(seln ? 1 : 0, 2) != 0;
        const bool twin = !isnew && ((lane >= 1 && (p1 | 1ull) == key && !(p1 & 1ull) && s1) ||
                                     (lane >= 2 && (p2 | 1ull) == key && !(p2 & 1ull) && s2));
        const bool cold = valid && !isnew && rold < C;
        const bool removed = cold && twin;
        const uint64_t mrem = ballot(removed);
        const uint32_t nnew = min(C, (uint32_t)__popcll(mnew));
        const uint32_t nold = min(C, (uint32_t)__popcll(mold)) - (uint32_t)__popcll(mrem);
        uint2* cs = v.cand + (size_t)u * 2 * C;
        const uint32_t id = (uint32_t)(key >> 1) & 0x7fffffffu;
        if (seln) {
            cs[rnew] = make_uint2(id, mpos);
            atomicAdd(&v.cap[mpos], nnew - 1 + nold);
        }
        if (cold && !removed) {
            cs[nnew + rold - mbcnt(mrem)] = make_uint2(id, mpos);
            if (nnew > 0) atomicAdd(&v.cap[mpos], nnew);
        }
        // forward NEW entries whose member was sampled new become OLD
        if (real && isnew && idx < (uint32_t)K && (seln || (dup && s1)))
            v.lpos[(size_t)u * K + idx] = mpos;
        if (lane == 0) v.nn[u] = nnew | (nold << 16);
    }
}

void launch_select(const Views& v, uint64_t st, hipStream_t s) {
    hipLaunchKernelGGL(k_select_small, dim3(grid_for(v.N, kSelWaves, 1 << 16)), dim3(256), 0, s, v, st);
    hipLaunchKernelGGL(k_select_large, dim3(1024), dim3(256), 0, s, v, st);
}

// ------------------------------------------------------------------ join (a3, a4)

// Append a proposal to the bucket of target position t. The capacity of each
// bucket bounds its proposals by construction; the check keeps a violated
// bound from writing outside it.
__device__ __forceinline__ void emit(const Views& v, uint32_t t, uint64_t key, uint32_t src) {
    const uint32_t slot = v.poff[t] + atomicAdd(&v.pcnt[t], 1u);
    if (slot < v.poff[t + 1]) {
        v.pkey[slot] = key;
        v.ppos[slot] = src;
    } else {
        atomicOr((unsigned long long*)&v.counters[kCntError], 2ull);
    }
}

constexpr int kJoinWaves = 4;

static inline size_t join_valu_wave_bytes(const Views& v) {
    const size_t m = 2 * (size_t)v.C;
    return m * v.dp * 4 + m * 16;
}

bool join_valu_fits(const Views& v) { return join_valu_wave_bytes(v) * kJoinWaves <= 64 * 1024; }

// Low-d local join: one wave per owner; member rows staged in LDS, one lane
// per (new member, member) cell; direct-form distances; each pair proposes
// both ways, filtered against the targets' snapshot K-th keys (a proposal not
// below that key can never enter the list).
__global__ __launch_bounds__(256) void k_join_valu(Views v) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int C2 = 2 * v.C, dp = v.dp, dp4 = dp >> 2, K = v.K;
    const double rdp4 = 1.0 / dp4;
    unsigned char* base = smem + (size_t)w * ((size_t)C2 * dp * 4 + (size_t)C2 * 16);
    float* rows = reinterpret_cast<float*>(base);
    uint64_t* thr = reinterpret_cast<uint64_t*>(base + (size_t)C2 * dp * 4);
    uint32_t* oid = reinterpret_cast<uint32_t*>(thr + C2);
    uint32_t* opos = oid + C2;
    for (int u = blockIdx.x * kJoinWaves + w; u < v.N; u += gridDim.x * kJoinWaves) {
        const uint32_t nn = v.nn[u];
        const int nnew = (int)(nn & 0xffffu), m = nnew + (int)(nn >> 16);
        if (nnew == 0) continue;
        const uint2* cs = v.cand + (size_t)u * C2;
        for (int i = lane; i < m; i += 64) {
            const uint2 c = cs[i];
            oid[i] = c.x;
            opos[i] = c.y;
            thr[i] = v.lkey[(size_t)c.y * K + K - 1];
        }
        wave_sync();
        for (int idx = lane; idx < m * dp4; idx += 64) {
            const int r = (int)udiv((uint32_t)idx, (uint32_t)dp4, rdp4), c = idx - r * dp4;
            reinterpret_cast<float4*>(rows)[idx] =
                reinterpret_cast<const float4*>(v.Xp + (size_t)opos[r] * dp)[c];
        }
        wave_sync();
        const int ncell = nnew * m;
        const double rm = 1.0 / m;
        for (int idx = lane; idx < ncell; idx += 64) {
            const int i = (int)udiv((uint32_t)idx, (uint32_t)m, rm), j = idx - i * m;
            if (j < nnew && j <= i) continue;
            const float D = dist_direct(rows + (size_t)i * dp, rows + (size_t)j * dp, dp);
            const uint64_t kb = (uint64_t)__float_as_uint(D) << 32;
            const uint64_t ki = kb | oid[j], kj = kb | oid[i];
            if (ki < thr[i]) emit(v, opos[i], ki, opos[j]);
            if (kj < thr[j]) emit(v, opos[j], kj, opos[i]);
        }
        wave_sync();
    }
}

void launch_join_valu(const Views& v, hipStream_t s) {
    const size_t lds = join_valu_wave_bytes(v) * kJoinWaves;
    hipLaunchKernelGGL(k_join_valu, dim3(grid_for(v.N, kJoinWaves, 1 << 16)), dim3(256), lds, s, v);
}

// High-d local join on FP32 MFMA (v_mfma_f32_16x16x4f32): per owner, the
// Gram tiles G = A B^T with B = [new | old] member rows and A = the new rows
// (tile rt of A is tile rt of B), only tiles (rt <= ct). Rows are read with
// 32-byte loads per lane: lane (c = lane%16, g = lane/16) holds dims
// [k0 + 8g, k0 + 8g + 8) of member 16*tile + c and feeds component q to
// instruction q. D = ||a||^2 + ||b||^2 - 2 a.b, clamped at 0.
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaMaxCT = 4;   // m = 2C <= 64

__global__ __launch_bounds__(256) void k_join_mfma(Views v) {
    __shared__ uint64_t s_thr[kJoinWaves][64];
    __shared__ uint32_t s_oid[kJoinWaves][64];
    __shared__ uint32_t s_pos[kJoinWaves][64];
    __shared__ float s_nrm[kJoinWaves][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int C2 = 2 * v.C, dp = v.dp, K = v.K;
    const int c16 = lane & 15, g = lane >> 4;
    for (int u = blockIdx.x * kJoinWaves + w; u < v.N; u += gridDim.x * kJoinWaves) {
        const uint32_t nn = v.nn[u];
        const int nnew = (int)(nn & 0xffffu), m = nnew + (int)(nn >> 16);
        if (nnew == 0) continue;
        const uint2* cs = v.cand + (size_t)u * C2;
        if (lane < m) {
            const uint2 c = cs[lane];
            s_oid[w][lane] = c.x;
            s_pos[w][lane] = c.y;
            s_thr[w][lane] = v.lkey[(size_t)c.y * K + K - 1];
            s_nrm[w][lane] = v.nrm[c.y];
        }
        wave_sync();
        const int RT = (nnew + 15) >> 4, CT = (m + 15) >> 4;
        const float* rp[kMfmaMaxCT];
        bool rv[kMfmaMaxCT];
        for (int ct = 0; ct < kMfmaMaxCT; ++ct) {
            const int j = ct * 16 + c16;
            rv[ct] = ct < CT && j < m;
            rp[ct] = v.Xp + (size_t)(rv[ct] ? s_pos[w][j] : 0u) * dp + g * 8;
        }
        floatx4 acc[kMfmaMaxCT * (kMfmaMaxCT + 1) / 2];
        for (int t = 0; t < kMfmaMaxCT * (kMfmaMaxCT + 1) / 2; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < dp; k0 += 32) {
            float f[kMfmaMaxCT][8];
            for (int ct = 0; ct < kMfmaMaxCT; ++ct) {
                if (rv[ct]) {
                    const float4 a = *reinterpret_cast<const float4*>(rp[ct] + k0);
                    const float4 b = *reinterpret_cast<const float4*>(rp[ct] + k0 + 4);
                    f[ct][0] = a.x; f[ct][1] = a.y; f[ct][2] = a.z; f[ct][3] = a.w;
                    f[ct][4] = b.x; f[ct][5] = b.y; f[ct][6] = b.z; f[ct][7] = b.w;
                } else {
                    for (int q = 0; q < 8; ++q) f[ct][q] = 0.f;
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                int t = 0;
#pragma unroll
                for (int rt = 0; rt < kMfmaMaxCT; ++rt)
#pragma unroll
                    for (int ct = rt; ct < kMfmaMaxCT; ++ct, ++t)
                        if (rt < RT && ct < CT)
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[rt][q], f[ct][q], acc[t], 0, 0, 0);
            }
        }
        // epilogue: lane holds rows 16rt + 4g + r, column 16ct + c16 of tile t
        int t = 0;
#pragma unroll
        for (int rt = 0; rt < kMfmaMaxCT; ++rt)
#pragma unroll
            for (int ct = rt; ct < kMfmaMaxCT; ++ct, ++t) {
                if (!(rt < RT && ct < CT)) continue;
                const int j = ct * 16 + c16;
                if (j >= m) continue;
                const uint32_t oj = s_oid[w][j], pj = s_pos[w][j];
                const uint64_t tj = s_thr[w][j];
                const float nj = s_nrm[w][j];
                for (int r = 0; r < 4; ++r) {
                    const int i = rt * 16 + g * 4 + r;
                    if (i >= nnew || (j < nnew && j <= i)) continue;
                    float D = (s_nrm[w][i] + nj) - 2.0f * acc[t][r];
                    D = D > 0.f ? D : 0.f;
                    const uint64_t kb = (uint64_t)__float_as_uint(D) << 32;
                    const uint64_t ki = kb | oj, kj = kb | s_oid[w][i];
                    if (ki < s_thr[w][i]) emit(v, s_pos[w][i], ki, pj);
                    if (kj < tj) emit(v, pj, kj, s_pos[w][i]);
                }
            }
        wave_sync();
    }
}

void launch_join_mfma(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_join_mfma, dim3(grid_for(v.N, kJoinWaves, 1 << 16)), dim3(256), 0, s, v);
}

// ------------------------------------------------------------------ merge (a5)

constexpr int kMergeWaves = 4;

// One wave per target with proposals. The list sits one entry per lane,
// ascending; lanes >= K hold +inf. Proposals are read 64 at a time and
// dropped when not below the current K-th key or when their id is in the
// snapshot list or already in the current list. A chunk with few survivors
// inserts them one by one (ballot rank, shift up); a larger one is sorted
// (bitonic), reversed and folded into the list with a lane-wise min, which
// leaves a bitonic sequence holding the 64 smallest keys, sorted again by one
// half-cleaner pass; equal keys (one id proposed by two owners) are then
// collapsed. Entries that enter are NEW; c_t counts ids not in the snapshot.
__global__ __launch_bounds__(256) void k_merge(Views v) {
    __shared__ uint64_t s_k[kMergeWaves][64];
    __shared__ uint32_t s_p[kMergeWaves][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int K = v.K;
    uint64_t changes = 0, props = 0;
    for (int p = blockIdx.x * kMergeWaves + w; p < v.N; p += gridDim.x * kMergeWaves) {
        const uint32_t base = v.poff[p];
        const uint32_t n = min(v.pcnt[p], v.poff[p + 1] - base);
        if (n == 0) continue;
        const size_t row = (size_t)p * K;
        uint64_t key = lane < K ? v.lkey[row + lane] : ~0ull;
        uint32_t pf = lane < K ? v.lpos[row + lane] : 0u;
        const uint32_t snap = lane < K ? (uint32_t)key : 0xffffffffu;
        uint64_t kth = rl64(key, K - 1);
        bool grown = false;  // list holds entries from proposals
        for (uint32_t c0 = 0; c0 < n; c0 += 64) {
            const uint32_t i = c0 + (uint32_t)lane;
            uint64_t pk = ~0ull;
            uint32_t pp = 0;
            if (i < n) {
                pk = v.pkey[base + i];
                pp = v.ppos[base + i] | kNewBit;
            }
            bool ok = pk < kth;
            if (__popcll(ballot(ok)) == 0) continue;
            const uint32_t pid = (uint32_t)pk;
            for (int k = 0; k < K; ++k) ok &= rl32(snap, k) != pid;
            if (grown) {
                const uint32_t cur = (uint32_t)key;
                for (int k = 0; k < K; ++k) ok &= rl32(cur, k) != pid;
            }
            uint64_t mask = ballot(ok);
            if (mask == 0) continue;
            grown = true;
            if (__popcll(mask) <= 4) {
                while (mask) {
                    const int j = __ffsll((long long)mask) - 1;
                    mask &= mask - 1;
                    const uint64_t x = rl64(pk, j);
                    if (x >= kth) continue;
                    if (ballot(lane < K && (uint32_t)key == (uint32_t)x)) continue;  // same id, same key
                    const uint32_t xp = rl32(pp, j);
                    const int at = __popcll(ballot(lane < K && key < x));
                    const uint64_t ku = shfl_up64(key, 1);
                    const uint32_t pu = (uint32_t)__shfl_up((int)pf, 1);
                    if (lane > at && lane < K) {
                        key = ku;
                        pf = pu;
                    }
                    if (lane == at) {
                        key = x;
                        pf = xp;
                    }
                    kth = rl64(key, K - 1);
                }
            } else {
                if (!ok) pk = ~0ull;
                wave_sort(pk, pp);
                const uint64_t rk = shfl64(pk, 63 - lane);
                const uint32_t rp = (uint32_t)__shfl((int)pp, 63 - lane);
                if (rk < key) {
                    key = rk;
                    pf = rp;
                }
                wave_bitonic_clean(key, pf);
                const uint64_t prevk = shfl_up64(key, 1);  // all lanes take part in the shuffle
                const bool dupk = lane > 0 && key != ~0ull && prevk == key;
                const uint64_t dm = ballot(dupk);
                if (dm) {
                    s_k[w][lane] = ~0ull;
                    wave_sync();
                    if (!dupk) {
                        const uint32_t to = (uint32_t)lane - mbcnt(dm);
                        s_k[w][to] = key;
                        s_p[w][to] = pf;
                    }
                    wave_sync();
                    key = s_k[w][lane];
                    pf = s_p[w][lane];
                    wave_sync();
                }
                if (lane >= K) {
                    key = ~0ull;
                    pf = 0u;
                }
                kth = rl64(key, K - 1);
            }
        }
        // an id twice in a row would mean two different keys for one pair
        bool twice = false;
        for (int k = 0; k < K; ++k) {
            const uint32_t ik = rl32((uint32_t)key, k);
            twice |= lane < K && k != lane && ik == (uint32_t)key;
        }
        if (ballot(twice) && lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 8ull);
        bool entered = lane < K;
        for (int k = 0; k < K; ++k) entered &= rl32(snap, k) != (uint32_t)key;
        if (lane < K) {
            v.lkey[row + lane] = key;
            v.lpos[row + lane] = pf;
        }
        changes += (uint64_t)__popcll(ballot(entered));
        props += n;
    }
    if (lane == 0 && (changes | props)) {
        atomicAdd((unsigned long long*)&v.counters[kCntChanges], (unsigned long long)changes);
        atomicAdd((unsigned long long*)&v.counters[kCntProposals], (unsigned long long)props);
    }
}

void launch_merge(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_merge, dim3(grid_for(v.N, kMergeWaves, 4096)), dim3(256), 0, s, v);
}

__global__ void k_finish_counters(Views v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) v.counters[kCntPairs2] = v.poff[v.N];
}

void launch_finish_counters(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_finish_counters, dim3(1), dim3(64), 0, s, v);
}

// ------------------------------------------------------------------ finalize (a8)

__global__ void k_finalize(Views v, int32_t* __restrict__ ids, float* __restrict__ dists, uint8_t* __restrict__ flags) {
    const int64_t NK = (int64_t)v.N * v.K;
    const double rk = 1.0 / v.K;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < NK; e += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)udiv((uint32_t)e, (uint32_t)v.K, rk), k = (int)(e - (int64_t)p * v.K);
        const int64_t o = (int64_t)v.orig[p] * v.K + k;
        const uint64_t key = v.lkey[e];
        if (ids) ids[o] = (int32_t)(uint32_t)key;
        if (dists) dists[o] = __uint_as_float((uint32_t)(key >> 32));
        if (flags) flags[o] = (v.lpos[e] & kNewBit) ? 1 : 0;
    }
}

void launch_finalize(const Views& v, int32_t* ids, float* dists, uint8_t* flags, hipStream_t s) {
    const int64_t NK = (int64_t)v.N * v.K;
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(NK, 256, 1 << 16)), dim3(256), 0, s, v, ids, dists, flags);
}

__global__ void k_export_samples(Views v, int32_t* __restrict__ dnew, int32_t* __restrict__ dold,
                                 int32_t* __restrict__ counts) {
    const int C = v.C;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < v.N; p += gridDim.x * blockDim.x) {
        const int o = v.orig[p];
        const uint32_t nn = v.nn[p];
        const int a = (int)(nn & 0xffffu), b = (int)(nn >> 16);
        const uint2* cs = v.cand + (size_t)p * 2 * C;
        for (int i = 0; i < C; ++i) {
            dnew[(size_t)o * C + i] = i < a ? (int32_t)cs[i].x : -1;
            dold[(size_t)o * C + i] = i < b ? (int32_t)cs[a + i].x : -1;
        }
        counts[2 * (size_t)o] = a;
        counts[2 * (size_t)o + 1] = b;
    }
}

void launch_export_samples(const Views& v, int32_t* dnew, int32_t* dold, int32_t* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_export_samples, dim3(grid_for(v.N, 256, 8192)), dim3(256), 0, s, v, dnew, dold, counts);
}

// ------------------------------------------------------------------ permutation (a7)

void launch_permute(const Views&, hipStream_t) {}

}  // namespace knng
