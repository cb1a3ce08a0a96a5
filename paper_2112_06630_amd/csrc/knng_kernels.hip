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
#include <climits>

#include <hip/hip_ext.h>

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

// Turbosampling coin (Sec. 3.1): an entry of weight wt among n entries of its
// flag passes with probability C/n, i.e. iff wt * n < C * 2^32 (exact).
__device__ __forceinline__ bool turbo_coin(uint32_t wt, uint32_t n, uint32_t C) {
    return (uint64_t)wt * n < ((uint64_t)C << 32);
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

// Value of lane (lane ^ m). Distances inside a row of 16 lanes use DPP moves
// in the vector ALU (quad permutations; row mirror i -> i^15 and half mirror
// i -> i^7 within a row, composed: 4 = half mirror then quad reverse (i^7^3),
// 8 = mirror then half mirror (i^15^7); 15 = the mirror alone); other
// distances go through the LDS crossbar. m is a compile-time constant after the sorting loops unroll.
__device__ __forceinline__ uint32_t xor_lanes(uint32_t x, int m) {
    switch (m) {
        case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
        case 4: {
            const int y = __builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, false);          // row_half_mirror
            return (uint32_t)__builtin_amdgcn_mov_dpp(y, 0x1B, 0xF, 0xF, false);              // quad_perm [3,2,1,0]
        }
        case 8: {
            const int y = __builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, false);          // row_mirror
            return (uint32_t)__builtin_amdgcn_mov_dpp(y, 0x141, 0xF, 0xF, false);             // row_half_mirror
        }
        case 15: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, false);  // row_mirror
        default: return (uint32_t)__shfl_xor((int)x, m);
    }
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x, int m) {
    const uint32_t lo = xor_lanes((uint32_t)x, m);
    const uint32_t hi = xor_lanes((uint32_t)(x >> 32), m);
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

// Value of another lane of the caller's 16-lane row, r lanes away with
// wrap-around (DPP row rotation): r = 1 .. 15 visit every other lane of the
// row once. r is a compile-time constant after unrolling. Callers that need
// to know which lane a value came from rotate the lane index alongside.
__device__ __forceinline__ uint32_t row_rot(uint32_t x, int r) {
    switch (r) {
        case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x121, 0xF, 0xF, false);   // row_ror
        case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x122, 0xF, 0xF, false);
        case 3: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x123, 0xF, 0xF, false);
        case 4: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x124, 0xF, 0xF, false);
        case 5: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x125, 0xF, 0xF, false);
        case 6: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x126, 0xF, 0xF, false);
        case 7: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x127, 0xF, 0xF, false);
        case 8: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, false);
        case 9: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x129, 0xF, 0xF, false);
        case 10: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x12A, 0xF, 0xF, false);
        case 11: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x12B, 0xF, 0xF, false);
        case 12: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x12C, 0xF, 0xF, false);
        case 13: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x12D, 0xF, 0xF, false);
        case 14: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x12E, 0xF, 0xF, false);
        case 15: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x12F, 0xF, 0xF, false);
        default: return x;
    }
}

// One compare-exchange step of a bitonic network across the wave: lanes
// lane and lane^j exchange; an ascending block keeps the smaller key in its
// lower lane. Equal keys are left in place.
__device__ __forceinline__ void cmpx(uint64_t& k, uint32_t& v, int j, bool asc) {
    const int lane = lane_id();
    const uint64_t ok = shfl_xor64(k, j);
    const uint32_t ov = xor_lanes(v, j);
    const bool low = (lane & j) == 0;
    // lane masks and selects, no branch: a conditional choice between the two
    // comparisons compiles to divergent control flow per stage
    const bool keep_min = asc == low;
    const bool lt = ok < k, gt = k < ok;
    const bool sw = (keep_min & lt) | (!keep_min & gt);
    k = sw ? ok : k;
    v = sw ? ov : v;
}

// Ascending bitonic sort of distinct 32-bit keys within segments of W lanes
// (W = 64: the whole wave; W = 32: lanes 0-31 and 32-63 separately).
template <int W>
__device__ __forceinline__ void seg_sort32(uint32_t& k) {
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= W; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) {
            const uint32_t o = xor_lanes(k, j);
            const bool keep_min = (size == W || (lane & size) == 0) == ((lane & j) == 0);
            k = keep_min ? min(k, o) : max(k, o);
        }
    }
}

// Odd-even transposition passes within W-lane segments on (key, value)
// pairs until a pass swaps nothing (the wave leaves together): finishes the
// order of a sequence that is already sorted up to short runs.
template <int W>
__device__ __forceinline__ void seg_fixup(uint64_t& key, uint32_t& val) {
    const int lane = lane_id(), sl = lane & (W - 1);
    for (int pass = 0; pass < W; ++pass) {
        bool any = false;
#pragma unroll
        for (int ph = 0; ph < 2; ++ph) {
            const bool lower = (sl & 1) == ph;    // phase 0: pairs (2i, 2i+1); phase 1: (2i+1, 2i+2)
            const bool has = lower ? sl + 1 < W : sl >= 1;
            const int partner = has ? (lower ? lane + 1 : lane - 1) : lane;
            const uint64_t ok = shfl64(key, partner);
            const uint32_t ov = (uint32_t)__shfl((int)val, partner);
            const bool sw = has && (lower ? ok < key : key < ok);
            key = sw ? ok : key;
            val = sw ? ov : val;
            any |= sw;
        }
        if (ballot(any) == 0ull) break;
    }
}

// Sorts a bitonic sequence of 64 pairs ascending.
__device__ __forceinline__ void wave_bitonic_clean(uint64_t& k, uint32_t& v) {
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) cmpx(k, v, j, true);
}

// An iteration enqueued ahead of the host's stop decision returns at once
// when the previous iteration met the stop rule.
__device__ __forceinline__ bool stopped(const Views& v) { return v.stop && *v.stop != 0u; }

// Sets `bits` in a device-wide flag word. Every wave of a pass may report the
// same bits; an atomic per wave on one address serialises at the cache (half
// a millisecond for 50000 waves), so the word is read first and the atomic
// issued only when a bit is still missing.
__device__ __forceinline__ void flag_or(uint64_t* word, uint64_t bits) {
    const uint64_t cur = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((cur & bits) != bits) atomicOr((unsigned long long*)word, (unsigned long long)bits);
}

// Batched form: position p belongs to dataset ds[p]; a single build has no
// dataset table and every position is active.
__device__ __forceinline__ bool pos_active(const Views& v, int p) { return !v.ds || v.active[v.ds[p]] != 0u; }

// Sample stream state of the owner's dataset for iteration t (t >= 1).
__device__ __forceinline__ uint64_t sample_state(const Views& v, int p, uint64_t st, int t) {
    return v.ds ? v.st_table[(size_t)(t - 1) * v.nds + v.ds[p]] : st;
}

// e(u): pairs an owner joins, new x new and new x old (Sec. 2).
__device__ __forceinline__ uint32_t owner_pairs(uint32_t nnew, uint32_t nold) {
    return nnew * (nnew - (nnew ? 1u : 0u)) / 2u + nnew * nold;
}

// First proposal slot of target p. Only the members of p's pool can sample p
// (the pool relation is symmetric: p is in pool(u) iff u is in pool(p)); there
// are at most K + rdeg(p) of them and each proposes to p at most 2C - 1 times
// (once per pair containing p), so bucket p holds (2C - 1)(K + rdeg(p))
// slots, and the buckets of positions 0..p-1 hold (2C - 1)(K p + roff[p]).
__device__ __forceinline__ uint32_t bucket_lo(const Views& v, int p) {
    return (uint32_t)(2 * v.C - 1) * ((uint32_t)v.K * (uint32_t)p + v.roff[p]);
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

// Squared differences of one 32-dimension chunk: four partial sums
// (components 0..3 of the eight 16-byte groups, in dimension order), added as
// (s0 + s1) + (s2 + s3).
__device__ __forceinline__ float chunk32_sq(const float4* __restrict__ pa, const float4* __restrict__ pb) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float4 x = pa[c], y = pb[c];
        const float t0 = x.x - y.x, t1 = x.y - y.y, t2 = x.z - y.z, t3 = x.w - y.w;
        s0 = fmaf(t0, t0, s0);
        s1 = fmaf(t1, t1, s1);
        s2 = fmaf(t2, t2, s2);
        s3 = fmaf(t3, t3, s3);
    }
    return (s0 + s1) + (s2 + s3);
}

// The precision form's stored distance: the chunk sums added into FP64 in
// chunk order and rounded to FP32 once (dp % 32 == 0). The rescore in the
// join computes the same value from rows staged in LDS.
__device__ __forceinline__ float dist_rescore(const float* __restrict__ a, const float* __restrict__ b, int dp) {
    double tot = 0.0;
    for (int k0 = 0; k0 < dp; k0 += 32)
        tot += (double)chunk32_sq(reinterpret_cast<const float4*>(a + k0), reinterpret_cast<const float4*>(b + k0));
    return (float)tot;
}

// q = a / b for 0 <= a < 2^31, 1 <= b, via a double reciprocal and one fix-up.
__device__ __forceinline__ uint32_t udiv(uint32_t a, uint32_t b, double rcp) {
    uint32_t q = (uint32_t)((double)a * rcp);
    if (q * b > a) --q;
    else if ((q + 1) * b <= a) ++q;
    return q;
}

// Items are split into 8 contiguous ranges, one per XCD: workgroups are
// dispatched round-robin over the 8 XCDs, so workgroup b runs on XCD b % 8,
// and owners that are close in storage order (after the graph-ordered
// permutation: close in the data space) then share one L2.
struct XcdRange {
    int next, end, step;
};

__device__ __forceinline__ XcdRange xcd_range(int n, int waves_per_block, int wave) {
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    // fewer workgroups than XCDs (a few dozen items): one grid-stride range
    if (G < 8) return XcdRange{b * waves_per_block + wave, n, G * waves_per_block};
    const int x = b & 7, bi = b >> 3;
    const int nbx = (G - x + 7) >> 3;           // workgroups on this XCD
    const int per = (n + 7) >> 3;               // items per XCD range
    const int lo = min(n, x * per), hi = min(n, lo + per);
    return XcdRange{lo + bi * waves_per_block + wave, hi, nbx * waves_per_block};
}

static inline int grid_for(int64_t items, int per_block, int cap = 1 << 20) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// Workgroup cap of the select and join passes (their loops stride over the
// owners, so any grid covers them).
static inline int pass_cap(const Views& v) { return v.grid_cap > 0 ? v.grid_cap : 1 << 16; }

// Launch with optional start / stop events recorded by the dispatch packet.
template <typename... P, typename... A>
static void launch_timed(void (*kernel)(P...), dim3 g, dim3 b, size_t lds, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1, A... args) {
    if (e0 || e1)
        hipExtLaunchKernelGGL(kernel, g, b, (uint32_t)lds, s, e0, e1, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, g, b, lds, s, args...);
}

// ------------------------------------------------------------------ fills

// A non-null `stop` word that is set skips the pass (a stopped batch group).
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n, const uint32_t* stop) {
    if (stop && *stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n, const uint32_t* stop) {
    if (stop && *stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s, const uint32_t* stop) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 1024, 4096)), dim3(256), 0, s, p, v, n, stop);
}

void launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s, const uint32_t* stop) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 1024, 4096)), dim3(256), 0, s, p, v, n, stop);
}

// ------------------------------------------------------------------ layout (a0)

// Rows padded to dp floats (zeros), identity permutation, finiteness check.
__global__ void k_pad_rows(const float* __restrict__ X, int N, int d, int dp, float* __restrict__ Xp,
                           int32_t* __restrict__ orig, int32_t* __restrict__ posof, uint64_t* counters,
                           RowKey* __restrict__ rk) {
    const int64_t total = (int64_t)N * dp;
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / dp;
        const int c = (int)(i - r * dp);
        const float x = c < d ? X[r * d + c] : 0.f;
        bad |= (__float_as_uint(x) & 0x7f800000u) == 0x7f800000u;
        Xp[i] = x;
        if (rk) reinterpret_cast<float*>(&rk[r].x)[c] = x;   // dp == 4 here
        if (c == 0) {
            orig[r] = (int32_t)r;
            posof[r] = (int32_t)r;
        }
    }
    if (bad) atomicOr((unsigned long long*)&counters[kCntNonFinite], 1ull);
}

void launch_pad_rows(const float* X, const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_rows, dim3(grid_for((int64_t)v.N * v.dp, 1024, 8192)), dim3(256), 0, s, X, v.N, v.d,
                       v.dp, v.Xp, v.orig, v.posof, v.counters, v.rk);
}

// Squared norms of padded rows, one wave per row, in the order k_prep uses
// (FP64 lane sums over j mod 4, then a fixed xor tree): one value per row
// whichever kernel laid the rows out.
__global__ __launch_bounds__(256) void k_norms(const float* __restrict__ Xp, int N, int dp, float* __restrict__ nrm,
                                               double* __restrict__ nrm64) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    for (int r = blockIdx.x * 4 + w; r < N; r += gridDim.x * 4) {
        const float* y = Xp + (size_t)r * dp;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int j = 4 * lane; j < dp; j += 256) {
            const float4 q = *reinterpret_cast<const float4*>(y + j);
            s0 = fma((double)q.x, (double)q.x, s0);
            s1 = fma((double)q.y, (double)q.y, s1);
            s2 = fma((double)q.z, (double)q.z, s2);
            s3 = fma((double)q.w, (double)q.w, s3);
        }
        double sn = (s0 + s1) + (s2 + s3);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sn += __shfl_xor(sn, o);
        if (lane == 0) {
            nrm64[r] = sn;
            nrm[r] = (float)sn;
        }
    }
}

void launch_norms(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_norms, dim3(grid_for(v.N, 4, 16384)), dim3(256), 0, s, v.Xp, v.N, v.dp, v.nrm, v.nrm64);
}

// ------------------------------------------------------------------ init (a1)

constexpr int kRowWaves = 4;

// Dot product of 8 consecutive dimensions (chunk c of a row) with the same
// dimensions of another row, FP32 products and sums in dimension order. The
// FP32 rows (two float4) and the one-plane BF16 rows (one uint4) give the
// same value whenever the FP32 values are exact in BF16, so a build that
// reads the plane and one that reads the FP32 rows agree bit for bit.
__device__ __forceinline__ float chunk_dot(const float4 a, const float4 b, float s) {
    s = fmaf(a.x, b.x, s);
    s = fmaf(a.y, b.y, s);
    s = fmaf(a.z, b.z, s);
    return fmaf(a.w, b.w, s);
}

__device__ __forceinline__ float chunk8_dot(const float4* __restrict__ a, const float4* __restrict__ b, int c,
                                            float s) {
    s = chunk_dot(a[2 * c], b[2 * c], s);
    return chunk_dot(a[2 * c + 1], b[2 * c + 1], s);
}

// byte rows: the same 8 products and sums in dimension order (every byte is
// exact in BF16 and FP32, so the value equals the BF16-plane one bit for bit)
__device__ __forceinline__ float chunk8_dot(const uint2* __restrict__ a, const uint2* __restrict__ b, int c,
                                            float s) {
    const uint2 x = a[c], y = b[c];
    const uint32_t av[2] = {x.x, x.y}, bv[2] = {y.x, y.y};
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k)
            s = fmaf((float)((av[q] >> (8 * k)) & 0xffu), (float)((bv[q] >> (8 * k)) & 0xffu), s);
    return s;
}

__device__ __forceinline__ float chunk8_dot(const uint4* __restrict__ a, const uint4* __restrict__ b, int c,
                                            float s) {
    const uint4 x = a[c], y = b[c];
    const uint32_t av[4] = {x.x, x.y, x.z, x.w}, bv[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        s = fmaf(__uint_as_float(av[q] << 16), __uint_as_float(bv[q] << 16), s);
        s = fmaf(__uint_as_float(av[q] & 0xffff0000u), __uint_as_float(bv[q] & 0xffff0000u), s);
    }
    return s;
}

// Gram-form distances of row u to the K rows pid (lane k < K holds pid of
// neighbour k), the wave streaming each row: lane l takes the 8-dimension
// chunks l, l + 64, ..., R rows at a time (byte rows: ten, so that K = 20
// takes two passes with more rows in flight; the value of each row does not
// depend on R); each row's lane sums are added by a fixed xor tree. Returns lane k's distance. T = float4 (FP32 rows,
// `stride` = d_pad / 4) or uint4 (one-plane BF16 rows, exact products,
// `stride` = d_pad / 8); `chunks` = d_pad / 8 either way.
template <typename T, int R = 4>
__device__ __forceinline__ float wave_gram_dists(const T* __restrict__ rows, int stride, int chunks, int u,
                                                 uint32_t pid, int K, const float* __restrict__ nrm) {
    const int lane = lane_id();
    const T* a = rows + (size_t)u * stride;
    float mine = 0.f;
    for (int k0 = 0; k0 < K; k0 += R) {
        const T* b[R];
#pragma unroll
        for (int q = 0; q < R; ++q) b[q] = rows + (size_t)rl32(pid, min(k0 + q, K - 1)) * stride;
        float s[R];
#pragma unroll
        for (int q = 0; q < R; ++q) s[q] = 0.f;
        for (int c = lane; c < chunks; c += 64) {
#pragma unroll
            for (int q = 0; q < R; ++q) s[q] = chunk8_dot(a, b[q], c, s[q]);
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s[q] += __shfl_xor(s[q], o);
            if (lane == k0 + q) {
                const float D = (nrm[u] + nrm[pid]) - 2.0f * s[q];
                mine = D > 0.f ? D : 0.f;
            }
        }
    }
    return mine;
}

// The same distances with FP64 products and sums and FP64 norms, rounded to
// FP32 once (data whose FP32 Gram sums are not exact).
__device__ __forceinline__ double chunk8_dot64(const float4* __restrict__ a, const float4* __restrict__ b, int c,
                                               double s) {
    const float4 x0 = a[2 * c], y0 = b[2 * c], x1 = a[2 * c + 1], y1 = b[2 * c + 1];
    s = fma((double)x0.x, (double)y0.x, s);
    s = fma((double)x0.y, (double)y0.y, s);
    s = fma((double)x0.z, (double)y0.z, s);
    s = fma((double)x0.w, (double)y0.w, s);
    s = fma((double)x1.x, (double)y1.x, s);
    s = fma((double)x1.y, (double)y1.y, s);
    s = fma((double)x1.z, (double)y1.z, s);
    return fma((double)x1.w, (double)y1.w, s);
}

__device__ __forceinline__ double chunk8_dot64(const uint4* __restrict__ a, const uint4* __restrict__ b, int c,
                                               double s) {
    const uint4 x = a[c], y = b[c];
    const uint32_t av[4] = {x.x, x.y, x.z, x.w}, bv[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        s = fma((double)__uint_as_float(av[q] << 16), (double)__uint_as_float(bv[q] << 16), s);
        s = fma((double)__uint_as_float(av[q] & 0xffff0000u), (double)__uint_as_float(bv[q] & 0xffff0000u), s);
    }
    return s;
}

// Short rows (at most 16 chunks): the wave splits into 64/P groups of P
// lanes (P = chunks rounded up to a power of two), one neighbour per group,
// one chunk per lane, and each group sums by the same xor steps the
// 64-lane tree takes once its upper steps have only added zeros: the same
// FP64 value, with 64/P neighbours per pass instead of 4.
template <typename T>
__device__ __forceinline__ float wave_gram_dists64(const T* __restrict__ rows, int stride, int chunks, int u,
                                                   uint32_t pid, int K, const double* __restrict__ nrm64) {
    const int lane = lane_id();
    const T* a = rows + (size_t)u * stride;
    float mine = 0.f;
    if (chunks <= 16) {
        int P = 1;
        while (P < chunks) P <<= 1;
        const int Q = 64 / P, q = lane / P, c = lane & (P - 1);
        for (int k0 = 0; k0 < K; k0 += Q) {
            const uint32_t pb = (uint32_t)__shfl((int)pid, min(k0 + q, K - 1));   // whole wave
            const T* b = rows + (size_t)pb * stride;
            double s = 0.0;
            if (c < chunks) s = chunk8_dot64(a, b, c, 0.0);
            for (int o = P >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o);
            const int j = lane - k0;   // lane k0 + j takes the sum of group j
            const double t = __shfl(s, (j >= 0 && j < Q) ? j * P : 0);
            if (j >= 0 && j < Q && lane < K) {
                const float D = (float)((nrm64[u] + nrm64[pid]) - 2.0 * t);
                mine = D > 0.f ? D : 0.f;
            }
        }
        return mine;
    }
    for (int k0 = 0; k0 < K; k0 += 4) {
        const T* b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = rows + (size_t)rl32(pid, min(k0 + q, K - 1)) * stride;
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int c = lane; c < chunks; c += 64) {
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] = chunk8_dot64(a, b[q], c, s[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s[q] += __shfl_xor(s[q], o);
            if (lane == k0 + q) {
                const float D = (float)((nrm64[u] + nrm64[pid]) - 2.0 * s[q]);
                mine = D > 0.f ? D : 0.f;
            }
        }
    }
    return mine;
}

// Lanes < K hold one entry each (position `pid` of the neighbour, NEW flag in
// pf). Computes D against row u, ranks the K keys and writes the sorted row.
// With `given` (a caller's state), the distances are taken as they are
// (given[u K + lane]) instead of computed, so that a state exported and
// loaded again keeps its keys bit for bit.
__device__ __forceinline__ void finish_row(const Views& v, int u, uint32_t pid, uint32_t pf, int mode,
                                           const float* given = nullptr) {
    const int lane = lane_id();
    const int K = v.K;
    uint64_t key = ~0ull;
    float Dg = 0.f;
    if (given) {
        if (lane < K) Dg = given[(size_t)u * K + lane];
    } else if (mode == kDistGram) {   // whole wave
        const bool plane = v.Xs && v.planes == 1;
        if (v.u8)
            Dg = wave_gram_dists<uint2, 10>(reinterpret_cast<const uint2*>(v.Xs + (size_t)v.N * v.dp), v.dp >> 3,
                                            v.dp >> 3, u, pid, K, v.nrm);
        else if (v.acc && plane)
            Dg = wave_gram_dists64(reinterpret_cast<const uint4*>(v.Xs), v.dp >> 3, v.dp >> 3, u, pid, K, v.nrm64);
        else if (v.acc)
            Dg = wave_gram_dists64(reinterpret_cast<const float4*>(v.Xp), v.dp >> 2, v.dp >> 3, u, pid, K, v.nrm64);
        else if (plane)
            Dg = wave_gram_dists(reinterpret_cast<const uint4*>(v.Xs), v.dp >> 3, v.dp >> 3, u, pid, K, v.nrm);
        else
            Dg = wave_gram_dists(reinterpret_cast<const float4*>(v.Xp), v.dp >> 2, v.dp >> 3, u, pid, K, v.nrm);
    }
    if (lane < K) {
        float D;
        if (given || mode == kDistGram) {
            D = Dg;
        } else {
            const float* a = v.Xp + (size_t)u * v.dp;
            const float* b = v.Xp + (size_t)pid * v.dp;
            D = v.Xb ? dist_rescore(a, b, v.dp) : dist_direct(a, b, v.dp);
        }
        key = key_of(D, (uint32_t)v.orig[pid]);
    }
    int rank = 0;
    for (int j = 0; j < K; ++j) rank += (rl64(key, j) < key) ? 1 : 0;
    if (lane < K) {
        v.lkey[(size_t)u * K + rank] = key;
        v.lpos[(size_t)u * K + rank] = pid | pf;
        if (rank == K - 1) {   // the joins read the record when there is one
            if (v.rk)
                v.rk[u].kth = key;
            else
                v.kth[u] = key;
        }
    }
}

// K distinct ids != u from H(seed,1,0,u,j), j = 0,1,...: the first K distinct
// draws in draw order, as in the oracle. Positions equal original ids here.
__global__ __launch_bounds__(256) void k_init(Views v, uint64_t st, int mode) {
    __shared__ uint32_t s_sel[kRowWaves][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int K = v.K;
    for (int u = blockIdx.x * kRowWaves + w; u < v.N; u += gridDim.x * kRowWaves) {
        // ids are local to the dataset (the whole build for a single one)
        uint32_t base = 0, n = (uint32_t)v.N;
        uint64_t sti = st;
        if (v.ds) {
            const uint32_t i = v.ds[u];
            base = v.dsbase[i];
            n = v.dsbase[i + 1] - base;
            sti = v.st_init[i];
        }
        const uint32_t ul = (uint32_t)u - base;
        int have = 0;
        for (uint32_t b0 = 0; have < K; b0 += 64) {
            const uint32_t j = b0 + (uint32_t)lane;
            const uint64_t h = mix64(sti ^ (((uint64_t)ul << 32) | j));
            uint32_t c = (uint32_t)(((h >> 32) * (uint64_t)(n - 1)) >> 32);
            c += (c >= ul) ? 1u : 0u;
            c += base;
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
        finish_row(v, u, pid, kNewBit, mode);
    }
}

// k_init for lists of at most 16 entries with direct-form distances: four
// points per wave, one per 16-lane row. Each row draws 16 ids at a time in
// draw order (the first K distinct draws are the same as k_init's 64 at a
// time), every lane then computes its entry's distance, and the entry's rank
// in the row comes from comparing keys around the row by rotation.
__global__ __launch_bounds__(256) void k_init_rows(Views v, uint64_t st) {
    __shared__ uint32_t s_sel[kRowWaves][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int sl = lane & 15, g0 = lane & ~15;
    const int K = v.K;
    uint32_t* sel = &s_sel[w][g0];
    for (int pb = (blockIdx.x * kRowWaves + w) * 4; pb < v.N; pb += gridDim.x * kRowWaves * 4) {
        const int u = pb + (lane >> 4);
        const bool valid = u < v.N;
        // ids are local to the dataset (the whole build for a single one)
        uint32_t base = 0, n = (uint32_t)v.N;
        uint64_t sti = st;
        if (valid && v.ds) {
            const uint32_t i = v.ds[u];
            base = v.dsbase[i];
            n = v.dsbase[i + 1] - base;
            sti = v.st_init[i];
        }
        const uint32_t ul = (uint32_t)u - base;
        int have = valid ? 0 : K;
        for (uint32_t b0 = 0; ballot(have < K) != 0ull; b0 += 16) {
            const uint32_t j = b0 + (uint32_t)sl;
            const uint64_t h = mix64(sti ^ (((uint64_t)ul << 32) | j));
            uint32_t c = (uint32_t)(((h >> 32) * (uint64_t)(n - 1)) >> 32);
            c += (c >= ul) ? 1u : 0u;
            c += base;
            bool novel = have < K;
            for (int i = 0; i < have; ++i) novel &= (sel[i] != c);
#pragma unroll
            for (int r = 1; r < 16; ++r) {   // an equal draw in a lower lane of the row comes first
                const uint32_t o = row_rot(c, r);
                const uint32_t ol = row_rot((uint32_t)sl, r);
                novel &= !(ol < (uint32_t)sl && o == c);
            }
            const uint64_t m = (ballot(novel) >> g0) & 0xffffull;
            const int rk = __popcll(m & ((1ull << sl) - 1));
            wave_sync();
            if (novel && have + rk < K) sel[have + rk] = c;
            wave_sync();
            have = min(K, have + __popcll(m));
        }
        const bool in = valid && sl < K;
        const uint32_t pid = in ? sel[sl] : 0u;
        wave_sync();
        uint64_t key = ~0ull;
        if (in) {
            const float* a = v.Xp + (size_t)u * v.dp;
            const float* b = v.Xp + (size_t)pid * v.dp;
            const float D = v.Xb ? dist_rescore(a, b, v.dp) : dist_direct(a, b, v.dp);
            key = key_of(D, (uint32_t)v.orig[pid]);
        }
        int rank = 0;
#pragma unroll
        for (int r = 1; r < 16; ++r) {
            const uint32_t lo = row_rot((uint32_t)key, r), hi = row_rot((uint32_t)(key >> 32), r);
            rank += ((((uint64_t)hi << 32) | lo) < key) ? 1 : 0;
        }
        if (in) {
            v.lkey[(size_t)u * K + rank] = key;
            v.lpos[(size_t)u * K + rank] = pid | kNewBit;
            if (rank == K - 1) {   // the joins read the record when there is one
                if (v.rk)
                    v.rk[u].kth = key;
                else
                    v.kth[u] = key;
            }
        }
    }
}

void launch_init(const Views& v, uint64_t st_init, int mode, hipStream_t s) {
    if (mode == kDistDirect && v.K <= 16)
        hipLaunchKernelGGL(k_init_rows, dim3(grid_for((v.N + 3) / 4, kRowWaves, 65536)), dim3(256), 0, s, v, st_init);
    else
        hipLaunchKernelGGL(k_init, dim3(grid_for(v.N, kRowWaves, 65536)), dim3(256), 0, s, v, st_init, mode);
}

// Load a caller state: ids are original ids (positions equal ids before any
// permutation); distances recomputed, rows re-sorted by key.
__global__ __launch_bounds__(256) void k_load_rows(Views v, const int32_t* __restrict__ ids,
                                                   const float* __restrict__ dists, const uint8_t* __restrict__ flags,
                                                   int mode) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    for (int u = blockIdx.x * kRowWaves + w; u < v.N; u += gridDim.x * kRowWaves) {
        uint32_t pid = 0, pf = 0;
        float D = 0.f;
        if (lane < v.K) {
            pid = (uint32_t)ids[(size_t)u * v.K + lane];
            pf = flags[(size_t)u * v.K + lane] ? kNewBit : 0u;
            if (dists) D = dists[(size_t)u * v.K + lane];
        }
        // a row must hold K distinct ids in [0, N), none equal to u, and
        // given distances must be finite and non-negative
        bool bad = lane < v.K && (pid >= (uint32_t)v.N || pid == (uint32_t)u || !(D >= 0.f && D < INFINITY));
        for (int j = 0; j < v.K; ++j) {
            const uint32_t pj = rl32(pid, j);
            bad |= lane < v.K && j != lane && pj == pid;
        }
        if (ballot(bad)) {
            if (lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 4ull);
            continue;
        }
        finish_row(v, u, pid, pf, mode, dists);
    }
}

void launch_load_rows(const Views& v, const int32_t* ids, const float* dists, const uint8_t* flags, int mode,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_load_rows, dim3(grid_for(v.N, kRowWaves, 65536)), dim3(256), 0, s, v, ids, dists, flags,
                       mode);
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
                                                    int n, uint32_t* __restrict__ bsum, const uint32_t* stop) {
    if (stop && *stop) return;
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

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ bsum, int nb, const uint32_t* stop) {
    if (stop && *stop) return;
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

__global__ void k_scan_add(uint32_t* __restrict__ out, int n, const uint32_t* __restrict__ bsum, int nb,
                           const uint32_t* stop) {
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += bsum[i / kScanBlock];
    if (i == 0) out[n] = bsum[nb];
}

void launch_scan(const uint32_t* in, uint32_t* out, int n, uint32_t* tmp, hipStream_t s, const uint32_t* stop) {
    const int nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_local, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, in, out, n, tmp, stop);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, nb > 0 ? nb : 1, stop);
    hipLaunchKernelGGL(k_scan_add, dim3((n + 256) / 256), dim3(256), 0, s, out, n, tmp, nb > 0 ? nb : 1, stop);
}

// ------------------------------------------------------------------ reverse lists (a2)

__global__ void k_rev_hist(Views v) {
    if (stopped(v)) return;
    const int64_t NK = (int64_t)v.N * v.K;
    const double rk = 1.0 / v.K;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < NK; e += (int64_t)gridDim.x * blockDim.x) {
        if (v.ds && !pos_active(v, (int)udiv((uint32_t)e, (uint32_t)v.K, rk))) continue;
        atomicAdd(&v.rdeg[v.lpos[e] & kPosMask], 1u);
    }
}

void launch_rev_hist(const Views& v, hipStream_t s, hipEvent_t e0) {
    const int64_t NK = (int64_t)v.N * v.K;
    launch_timed(k_rev_hist, dim3(grid_for(NK, 256, 1 << 16)), dim3(256), 0, s, e0, nullptr, v);
}

// Each edge u->v (flag f) becomes the reverse entry {w, orig u, pos u | f} of v.
__global__ void k_rev_scatter(Views v, uint64_t st0, int t) {
    if (stopped(v)) return;
    const int64_t NK = (int64_t)v.N * v.K;
    const double rk = 1.0 / v.K;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < NK; e += (int64_t)gridDim.x * blockDim.x) {
        const int u = (int)udiv((uint32_t)e, (uint32_t)v.K, rk);
        if (v.ds && !pos_active(v, u)) continue;
        const uint64_t st = sample_state(v, u, st0, t);
        const uint32_t pf = v.lpos[e];
        const uint32_t tp = pf & kPosMask;
        const uint32_t ov = (uint32_t)v.lkey[e];
        const uint32_t ou = (uint32_t)v.orig[u];
        const uint32_t w = pair_weight(st, ou, ov);
        const uint32_t slot = v.roff[tp] + atomicAdd(&v.rcur[tp], 1u);
        v.rev[slot] = make_uint4(w, ou, (uint32_t)u | (pf & kNewBit), 0u);
    }
}

void launch_rev_scatter(const Views& v, uint64_t st, int t, hipStream_t s) {
    const int64_t NK = (int64_t)v.N * v.K;
    hipLaunchKernelGGL(k_rev_scatter, dim3(grid_for(NK, 256, 1 << 16)), dim3(256), 0, s, v, st, t);
}

// Reverse lists by a counting sort with block-private counters (no global
// atomics). Targets are grouped in super-buckets of R = 2^shift consecutive
// positions. (1) each block counts its chunk of E list entries per
// super-bucket in LDS -> H[s][b]; (2) exclusive scan of H (s-major) gives each
// (super-bucket, block) its output range, and the start of super-bucket s is
// the number of entries with smaller targets; (3) each block writes its
// entries (target, w, source) into those ranges of a staging array; (4) one
// block per super-bucket counts its targets in LDS, writes their bucket
// offsets roff and places the entries. Orders inside a range depend on LDS
// atomic order only, and every reader of a bucket sorts it by key.
__global__ __launch_bounds__(1024) void k_rev_count(Views v) {
    if (stopped(v)) return;
    extern __shared__ uint32_t s_cnt[];
    const int S = v.rev_S, B = gridDim.x;
    const int64_t NK = (int64_t)v.N * v.K;
    const int64_t e0 = (int64_t)blockIdx.x * v.rev_E, e1 = min(NK, e0 + v.rev_E);
    for (int i = threadIdx.x; i < S; i += blockDim.x) s_cnt[i] = 0u;
    __syncthreads();
    const double rk = 1.0 / v.K;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        if (v.ds && !pos_active(v, (int)udiv((uint32_t)e, (uint32_t)v.K, rk))) continue;
        atomicAdd(&s_cnt[(v.lpos[e] & kPosMask) >> v.rev_shift], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < S; i += blockDim.x) v.rev_h[(size_t)i * B + blockIdx.x] = s_cnt[i];
}

__global__ __launch_bounds__(1024) void k_rev_part(Views v, uint64_t st0, int t) {
    if (stopped(v)) return;
    extern __shared__ uint32_t s_cur[];
    const int S = v.rev_S, B = gridDim.x;
    const int64_t NK = (int64_t)v.N * v.K;
    const int64_t e0 = (int64_t)blockIdx.x * v.rev_E, e1 = min(NK, e0 + v.rev_E);
    for (int i = threadIdx.x; i < S; i += blockDim.x) s_cur[i] = v.rev_hs[(size_t)i * B + blockIdx.x];
    __syncthreads();
    const double rk = 1.0 / v.K;
    uint4* stage = reinterpret_cast<uint4*>(v.pkey);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int u = (int)udiv((uint32_t)e, (uint32_t)v.K, rk);
        if (v.ds && !pos_active(v, u)) continue;
        const uint64_t st = sample_state(v, u, st0, t);
        const uint32_t pf = v.lpos[e];
        const uint32_t tp = pf & kPosMask;
        const uint32_t ou = (uint32_t)v.orig[u];
        const uint32_t w = pair_weight(st, ou, (uint32_t)v.lkey[e]);
        const uint32_t slot = atomicAdd(&s_cur[tp >> v.rev_shift], 1u);
        stage[slot] = make_uint4(tp, w, ou, (uint32_t)u | (pf & kNewBit));
    }
}

__global__ __launch_bounds__(1024) void k_rev_bucket(Views v) {
    if (stopped(v)) return;
    extern __shared__ uint32_t s_loc[];   // [R] counts, then cursors
    __shared__ uint32_t s_w[16];
    const int R = 1 << v.rev_shift, B = v.rev_B;
    const int sb = blockIdx.x, t = threadIdx.x, lane = lane_id(), w = t >> 6;
    const uint32_t lo = (uint32_t)sb << v.rev_shift;
    const uint32_t a = v.rev_hs[(size_t)sb * B], b = v.rev_hs[(size_t)(sb + 1) * B];
    const uint4* stage = reinterpret_cast<const uint4*>(v.pkey);
    for (int i = t; i < R; i += 1024) s_loc[i] = 0u;
    __syncthreads();
    for (uint32_t e = a + t; e < b; e += 1024) atomicAdd(&s_loc[stage[e].x - lo], 1u);
    __syncthreads();
    // exclusive scan of the R counts: each thread owns R/1024 consecutive ones
    const int per = R >> 10 > 0 ? R >> 10 : 1;
    const int i0 = t * per;
    uint32_t sum = 0;
    for (int q = 0; q < per; ++q)
        if (i0 + q < R) sum += s_loc[i0 + q];
    const uint32_t inc = wave_incl_scan(sum);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t run = a + inc - sum;
    for (int i = 0; i < w; ++i) run += s_w[i];
    for (int q = 0; q < per; ++q) {
        const int i = i0 + q;
        if (i < R) {
            const uint32_t c = s_loc[i];
            if (lo + (uint32_t)i < (uint32_t)v.N) v.roff[lo + i] = run;
            s_loc[i] = run;
            run += c;
        }
    }
    if (sb == (int)gridDim.x - 1 && t == 0) v.roff[v.N] = b;
    __syncthreads();
    for (uint32_t e = a + t; e < b; e += 1024) {
        const uint4 x = stage[e];
        const uint32_t slot = atomicAdd(&s_loc[x.x - lo], 1u);
        v.rev[slot] = make_uint4(x.y, x.z, x.w, 0u);
    }
}

void launch_rev_partition(const Views& v, uint64_t st, int t, hipStream_t s, hipEvent_t e0) {
    const size_t lds_s = (size_t)v.rev_S * 4;
    launch_timed(k_rev_count, dim3(v.rev_B), dim3(1024), lds_s, s, e0, nullptr, v);
    launch_scan(v.rev_h, v.rev_hs, v.rev_S * v.rev_B, v.rev_tmp, s, v.stop);
    hipLaunchKernelGGL(k_rev_part, dim3(v.rev_B), dim3(1024), lds_s, s, v, st, t);
    hipLaunchKernelGGL(k_rev_bucket, dim3(v.rev_S), dim3(1024), ((size_t)4 << v.rev_shift), s, v);
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
__global__ __launch_bounds__(256) void k_select_large(Views v, uint64_t st0, int t) {
    if (stopped(v)) return;
    __shared__ SelLds L;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int K = v.K, C = v.C;
    uint64_t* skey = L.key[w];
    uint32_t* spos = L.pos[w];
    for (int u = blockIdx.x * kSelWaves + w; u < v.N; u += gridDim.x * kSelWaves) {
        if (!v.big[u]) continue;
        const uint64_t st = sample_state(v, u, st0, t);
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
        // ---- turbosampling: pool entries per flag, with multiplicity ----
        uint32_t tot[2] = {0u, 0u};
        if (v.turbo) {
            for (int i0 = 0; i0 < P; i0 += 64) {
                const int i = i0 + lane;
                uint32_t pf = 0;
                if (i < P) pf = i < K ? v.lpos[(size_t)u * K + i] : v.rev[rb + (uint32_t)(i - K)].z;
                tot[0] += (uint32_t)__popcll(ballot(i < P && (pf & kNewBit)));
                tot[1] += (uint32_t)__popcll(ballot(i < P && !(pf & kNewBit)));
            }
        }
        // an entry's coin (staged key: old << 63 | w << 31 | id); the entries
        // that pass are a prefix of their flag's ranks
        auto coin = [&](uint64_t k) {
            return !v.turbo || turbo_coin((uint32_t)(k >> 31), tot[k >> 63], (uint32_t)C);
        };
        // ---- ranks among distinct keys; twin = NEW entry of the same member ----
        uint32_t nvnew = 0, ncnew = 0, ncold = 0;
        for (int i0 = 0; i0 < n; i0 += 64) {
            const int i = i0 + lane;
            const bool valid = i < n && !L.dup[w][i];
            const uint64_t ki = i < n ? skey[i] : ~0ull;
            const bool c = valid && coin(ki);
            nvnew += __popcll(ballot(valid && !(ki >> 63)));
            ncnew += __popcll(ballot(c && !(ki >> 63)));
            ncold += __popcll(ballot(c && (ki >> 63)));
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
        const uint32_t nnew = min((uint32_t)C, ncnew);
        // ---- old entries whose member is sampled as new are removed ----
        for (int i = lane; i < n; i += 64) {
            if (L.dup[w][i] || !(skey[i] >> 63)) continue;
            const uint32_t ro = L.rank[w][i] - nvnew;
            if (ro >= (uint32_t)C || !coin(skey[i])) continue;
            const int tw = L.twin[w][i];
            if (tw >= 0 && L.rank[w][tw] < (uint32_t)C && coin(skey[tw]))
                atomicOr((unsigned long long*)&L.oldmask[w], 1ull << ro);
        }
        wave_sync();
        const uint64_t omask = L.oldmask[w];
        const uint32_t nold = min((uint32_t)C, ncold) - (uint32_t)__popcll(omask);
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
                if (rank < (uint32_t)C && coin(ki)) {
                    cs[rank] = make_uint2(id, pos);
                    if (i < nf) v.lpos[(size_t)u * K + L.src[w][i]] = pos;  // flip NEW -> OLD
                }
            } else {
                const uint32_t ro = rank - nvnew;
                if (ro < (uint32_t)C && coin(ki) && !((omask >> ro) & 1ull)) {
                    const uint32_t slot = nnew + ro - (uint32_t)__popcll(omask & ((1ull << ro) - 1ull));
                    cs[slot] = make_uint2(id, pos);
                }
            }
        }
        if (lane == 0) {
            v.nn[u] = nnew | (nold << 16);
            v.cap[u] = owner_pairs(nnew, nold);
        }
        wave_sync();
    }
}

// Large pools when 2C <= 64: per flag, a weight threshold T is searched so
// that between 2C (>= C distinct members, as a member appears at most twice)
// and 64 entries of that flag have w <= T; those are gathered into one lane
// each and sorted like a small pool. Each search step is one ballot-count
// pass over the pool. OLD entries whose member was sampled NEW are removed
// by comparing with the (at most C) sampled new ids.
__device__ __forceinline__ uint64_t sel_key(uint32_t wt, uint32_t id, uint32_t pf) {
    return ((uint64_t)wt << 32) | ((uint64_t)id << 1) | ((pf & kNewBit) ? 0u : 1u);
}

__device__ __forceinline__ void pool_read(const Views& v, uint64_t st, int u, uint32_t ou, uint32_t rb, int i,
                                          uint32_t& wt, uint32_t& id, uint32_t& pf) {
    if (i < v.K) {
        const size_t e = (size_t)u * v.K + i;
        id = (uint32_t)v.lkey[e];
        pf = v.lpos[e];
        wt = pair_weight(st, ou, id);
    } else {
        const uint4 r = v.rev[rb + (uint32_t)(i - v.K)];
        wt = r.x;
        id = r.y;
        pf = r.z;
    }
}

// One owner whose pool has more than 64 entries (s_key, s_idx: 64 LDS slots
// of the calling wave).
// Pool entry i without its weight: member id and position word.
__device__ __forceinline__ void pool_ids(const Views& v, int u, uint32_t rb, int i, uint32_t& id, uint32_t& pf) {
    if (i < v.K) {
        const size_t e = (size_t)u * v.K + i;
        id = (uint32_t)v.lkey[e];
        pf = v.lpos[e];
    } else {
        const uint4 r = v.rev[rb + (uint32_t)(i - v.K)];
        id = r.y;
        pf = r.z;
    }
}

constexpr int kThrCache = 512;   // pool entries whose weight and flag a wave keeps in LDS

// Weight and flag (1: OLD) of pool entry i: from the LDS cache when the pool
// fits it, else read again (the hash recomputed for forward entries).
__device__ __forceinline__ void pool_wf(const Views& v, uint64_t st, int u, uint32_t ou, uint32_t rb, int i,
                                        bool cached, const uint32_t* c_wt, const uint8_t* c_old, uint32_t& wt,
                                        uint32_t& old) {
    if (cached) {
        wt = c_wt[i];
        old = c_old[i];
    } else {
        uint32_t id, pf;
        pool_read(v, st, u, ou, rb, i, wt, id, pf);
        old = (pf & kNewBit) ? 0u : 1u;
    }
}

// One owner whose pool has more than 64 entries (s_key, s_idx: 64 LDS slots
// of the calling wave; c_wt, c_old: kThrCache-entry cache of the weights and
// OLD flags). The threshold search and the gathers read the cache; only the
// survivors' ids are read again.
__device__ void select_large_thr_owner(const Views& v, uint64_t st, int u, uint32_t rb, int P, uint32_t ou,
                                       uint64_t* s_key, uint32_t* s_idx, uint32_t* c_wt, uint8_t* c_old) {
    const int lane = lane_id();
    const int K = v.K;
    const uint32_t C = (uint32_t)v.C;
    const bool cached = P <= kThrCache;
    uint32_t tot[2] = {0u, 0u};
    for (int i0 = 0; i0 < P; i0 += 64) {
        const int i = i0 + lane;
        uint32_t wt = 0, id = 0, pf = 0;
        if (i < P) {
            pool_read(v, st, u, ou, rb, i, wt, id, pf);
            if (cached) {
                c_wt[i] = wt;
                c_old[i] = (pf & kNewBit) ? 0u : 1u;
            }
        }
        tot[0] += __popcll(ballot(i < P && (pf & kNewBit)));
        tot[1] += __popcll(ballot(i < P && !(pf & kNewBit)));
    }
    wave_sync();
    uint32_t newid = 0xffffffffu;  // lane r < nnew: id of the sampled new member of rank r
    uint32_t nnew = 0, nold = 0;
    uint32_t flip_idx = 0xffffffffu, flip_pos = 0;
    uint2* cs = v.cand + (size_t)u * 2 * C;
    bool failed = false;
    for (int f = 0; f < 2; ++f) {
        // ---- threshold ----
        uint32_t T = 0xffffffffu;
        if (tot[f] > 64) {
            const uint32_t need = 2 * C;
            uint64_t lo = 0, hi = 0xffffffffull;
            uint64_t t = ((uint64_t)((need + 64) / 2) << 32) / tot[f];
            bool found = false;
            for (int it = 0; it < 48 && !found; ++it) {
                uint32_t cnt = 0;
                for (int i0 = 0; i0 < P; i0 += 64) {
                    const int i = i0 + lane;
                    uint32_t wt = 0, old = 2u;
                    if (i < P) pool_wf(v, st, u, ou, rb, i, cached, c_wt, c_old, wt, old);
                    cnt += __popcll(ballot(old == (uint32_t)f && wt <= (uint32_t)t));
                }
                if (cnt >= need && cnt <= 64) {
                    found = true;
                } else {
                    if (cnt < need) lo = t; else hi = t;
                    t = lo + (hi - lo) / 2;
                    if (hi - lo <= 1) break;
                }
            }
            if (!found) {
                failed = true;
                break;
            }
            T = (uint32_t)t;
        }
        // ---- gather the survivors of flag f ----
        uint32_t n = 0;
        s_key[lane] = ~0ull;
        wave_sync();
        for (int i0 = 0; i0 < P; i0 += 64) {
            const int i = i0 + lane;
            uint32_t wt = 0, old = 2u;
            if (i < P) pool_wf(v, st, u, ou, rb, i, cached, c_wt, c_old, wt, old);
            const bool surv = old == (uint32_t)f && wt <= T;
            const uint64_t m = ballot(surv);
            const uint32_t slot = n + mbcnt(m);
            if (surv && slot < 64) {
                uint32_t id, pf;
                pool_ids(v, u, rb, i, id, pf);
                s_key[slot] = sel_key(wt, id, pf);
                s_idx[slot] = (uint32_t)i;
            }
            n += (uint32_t)__popcll(m);
        }
        wave_sync();
        if (n > 64) {
            failed = true;
            break;
        }
        uint64_t key = s_key[lane];
        uint32_t idx = (uint32_t)lane < n ? s_idx[lane] : 0xffffffffu;
        wave_sync();
        {   // sort a distinct 32-bit proxy, fetch the full keys, finish equal-weight runs
            uint32_t x = (uint32_t)lane < n ? (((uint32_t)(key >> 32) & ~127u) | ((uint32_t)(key & 1ull) << 6) |
                                                (uint32_t)lane)
                                             : 0xffffffffu;
            seg_sort32<64>(x);
            const int src = (int)(x & 63u);
            const uint64_t fk = shfl64(key, src);
            const uint32_t fi = (uint32_t)__shfl((int)idx, src);
            key = (uint32_t)lane < n ? fk : ~0ull;
            idx = (uint32_t)lane < n ? fi : 0xffffffffu;
            seg_fixup<64>(key, idx);
        }
        const uint64_t p1 = shfl_up64(key, 1);
        const bool real = key != ~0ull;
        const bool dup = real && lane >= 1 && p1 == key;
        const bool valid = real && !dup;
        const uint64_t mv = ballot(valid);
        const uint32_t r = mbcnt(mv);
        const uint32_t id = (uint32_t)(key >> 1) & 0x7fffffffu;
        const bool coin = !v.turbo || turbo_coin((uint32_t)(key >> 32), tot[f], C);
        uint32_t pos = 0;
        if (valid && r < C && coin) {
            uint32_t wt2, id2, pf2;
            pool_read(v, st, u, ou, rb, (int)idx, wt2, id2, pf2);
            pos = pf2 & kPosMask;
        }
        if (f == 0) {
            const bool sel = valid && r < C && coin;
            const int s1 = __shfl_up(sel ? 1 : 0, 1);
            nnew = (uint32_t)__popcll(ballot(sel));
            if (sel) cs[r] = make_uint2(id, pos);
            // forward NEW entries of sampled members flip to OLD once the OLD
            // pass (which reads the flags as sampled) is done; the forward copy
            // may be the duplicate (second) one
            if (idx < (uint32_t)K && (sel || (dup && s1))) {
                uint32_t wt2, id2, pf2;
                pool_read(v, st, u, ou, rb, (int)idx, wt2, id2, pf2);
                flip_idx = idx;
                flip_pos = pf2 & kPosMask;
            }
            // sampled new ids to lanes 0..nnew-1 (they are the first valid lanes in order)
            s_idx[lane] = 0xffffffffu;
            wave_sync();
            if (sel) s_idx[r] = id;
            wave_sync();
            newid = s_idx[lane];
            wave_sync();
        } else {
            bool innew = false;
            for (uint32_t k = 0; k < nnew; ++k) {
                const uint32_t nk = rl32(newid, (int)k);
                innew |= nk == id;
            }
            const bool cand_old = valid && r < C && coin;
            const bool removed = cand_old && innew;
            const uint64_t mrem = ballot(removed);
            nold = (uint32_t)__popcll(ballot(cand_old)) - (uint32_t)__popcll(mrem);
            if (cand_old && !removed) cs[nnew + r - mbcnt(mrem)] = make_uint2(id, pos);
        }
    }
    if (failed) {   // reported; the owner samples nothing (its join is skipped)
        if (lane == 0) {
            atomicOr((unsigned long long*)&v.counters[kCntError], 16ull);
            v.nn[u] = 0u;
            v.cap[u] = 0u;
        }
        return;
    }
    if (flip_idx != 0xffffffffu) v.lpos[(size_t)u * K + flip_idx] = flip_pos;
    if (lane == 0) {
        v.nn[u] = nnew | (nold << 16);
        v.cap[u] = owner_pairs(nnew, nold);
    }
    wave_sync();
}

// Pool of one owner per W-lane segment (u, P: the segment's owner and pool
// size, P <= W; u == N: no owner), one entry per lane, in registers. Select
// key (w << 32) | (id << 1) | old: sorting it puts the two copies of a
// member reached by both routes with the same flag next to each other (the
// second is a duplicate), and a member's NEW entry right before its OLD
// entry. Ranks per flag are ballot prefix counts over the segment's sorted
// lanes. pool_load reads the entries (pos: the entry's position word).
template <int W>
__device__ __forceinline__ void pool_load(const Views& v, uint64_t st0, int t, int u, int P, uint64_t& key,
                                          uint32_t& pos) {
    const int sl = lane_id() & (W - 1);
    const int K = v.K;
    key = ~0ull;
    pos = 0;
    if (sl < P) {
        const uint32_t rb = v.roff[u];
        uint32_t id, pf, wt;
        if (sl < K) {
            const size_t e = (size_t)u * K + sl;
            id = (uint32_t)v.lkey[e];
            pf = v.lpos[e];
            wt = pair_weight(sample_state(v, u, st0, t), (uint32_t)v.orig[u], id);
        } else {
            const uint4 r = v.rev[rb + (uint32_t)(sl - K)];
            wt = r.x;
            id = r.y;
            pf = r.z;
        }
        key = ((uint64_t)wt << 32) | ((uint64_t)id << 1) | ((pf & kNewBit) ? 0u : 1u);
        pos = pf & kPosMask;
    }
}

// Sort key of the proxy order: top 25 weight bits, the OLD bit, the entry's
// lane in the segment (distinct, and in the select key's order wherever the
// top weight bits differ). Padding lanes take the largest value; a real
// proxy can equal it only in a full segment, so after the sort the first P
// lanes hold the entries.
template <int W>
__device__ __forceinline__ uint32_t pool_proxy(uint64_t key, int P) {
    const int sl = lane_id() & (W - 1);
    return sl < P ? (((uint32_t)(key >> 32) & ~127u) | ((uint32_t)(key & 1ull) << 6) | (uint32_t)sl) : 0xffffffffu;
}

// After the proxy sort: fetch the full keys, then finish the order of the
// rare runs of equal proxy weights on the full key. idx: source lane.
template <int W>
__device__ __forceinline__ void pool_unproxy(uint32_t k32, int P, uint64_t& key, uint32_t& idx) {
    const int lane = lane_id(), sl = lane & (W - 1);
    idx = (uint32_t)(lane & ~(W - 1)) | (k32 & (uint32_t)(W - 1));
    const uint64_t fk = shfl64(key, (int)idx);   // every lane takes part in the exchange
    key = sl < P ? fk : ~0ull;
    seg_fixup<W>(key, idx);
}

// Ranks, the new/old samples and the flips of one owner per segment, from
// its pool sorted by select key (key, source lane idx, positions pos by
// source lane).
template <int W>
__device__ __forceinline__ void pool_finish(const Views& v, int u, uint64_t key, uint32_t idx, uint32_t pos) {
    const int lane = lane_id(), sl = lane & (W - 1);
    const uint64_t seg = W == 64 ? ~0ull : (lane < 32 ? 0x00000000ffffffffull : 0xffffffff00000000ull);
    const int N = v.N, K = v.K;
    const uint32_t C = (uint32_t)v.C;
    const uint32_t mpos = (uint32_t)__shfl((int)pos, (int)idx);
    const uint64_t p1 = shfl_up64(key, 1), p2 = shfl_up64(key, 2);
    const bool real = key != ~0ull;
    const bool dup = real && sl >= 1 && p1 == key;
    const bool valid = real && !dup;
    const bool isnew = (key & 1ull) == 0;
    const uint64_t mnew = ballot(valid && isnew) & seg, mold = ballot(valid && !isnew) & seg;
    const uint32_t rnew = mbcnt(mnew), rold = mbcnt(mold);
    // turbosampling: the entry's coin against its flag's pool count (with
    // multiplicity); survivors are a prefix of the flag's ranks
    bool coin = true;
    if (v.turbo) {
        const uint32_t nf = (uint32_t)__popcll(ballot(real && isnew) & seg);
        const uint32_t no = (uint32_t)__popcll(ballot(real && !isnew) & seg);
        coin = turbo_coin((uint32_t)(key >> 32), isnew ? nf : no, C);
    }
    const bool seln = valid && isnew && rnew < C && coin;
    const bool s1 = __shfl_up(seln ? 1 : 0, 1) != 0, s2 = __shfl_up(seln ? 1 : 0, 2) != 0;
    const bool twin = !isnew && ((sl >= 1 && (p1 | 1ull) == key && !(p1 & 1ull) && s1) ||
                                 (sl >= 2 && (p2 | 1ull) == key && !(p2 & 1ull) && s2));
    const bool cold = valid && !isnew && rold < C && coin;
    const bool removed = cold && twin;
    const uint64_t mrem = ballot(removed) & seg;
    const uint32_t nnew = (uint32_t)__popcll(ballot(seln) & seg);
    const uint32_t nold = (uint32_t)__popcll(ballot(cold) & seg) - (uint32_t)__popcll(mrem);
    const uint32_t ei = idx & (W - 1);
    if (u < N) {
        uint2* cs = v.cand + (size_t)u * 2 * C;
        const uint32_t id = (uint32_t)(key >> 1) & 0x7fffffffu;
        if (seln) cs[rnew] = make_uint2(id, mpos);
        if (cold && !removed) cs[nnew + rold - mbcnt(mrem)] = make_uint2(id, mpos);
        // forward NEW entries whose member was sampled new become OLD
        if (real && isnew && ei < (uint32_t)K && (seln || (dup && s1)))
            v.lpos[(size_t)u * K + ei] = mpos;
        if (sl == 0) {
            v.nn[u] = nnew | (nold << 16);
            v.cap[u] = owner_pairs(nnew, nold);
        }
    }
}

template <int W>
__device__ __forceinline__ void select_pool(const Views& v, uint64_t st0, int t, int u, int P) {
    uint64_t key;
    uint32_t pos, idx;
    pool_load<W>(v, st0, t, u, P, key, pos);
    uint32_t k32 = pool_proxy<W>(key, P);
    seg_sort32<W>(k32);
    pool_unproxy<W>(k32, P, key, idx);
    pool_finish<W>(v, u, key, idx, pos);
}

// Two owners of pools of at most 64 entries in one wave, one after the other
// in registers: their loads are issued together and their sorts interleaved
// stage by stage, so the two dependency chains overlap.
__device__ __forceinline__ void select_pool_x2(const Views& v, uint64_t st0, int t, int ua, int Pa, int ub, int Pb) {
    uint64_t ka, kb;
    uint32_t pa, pb, ia, ib;
    pool_load<64>(v, st0, t, ua, Pa, ka, pa);
    pool_load<64>(v, st0, t, ub, Pb, kb, pb);
    uint32_t xa = pool_proxy<64>(ka, Pa), xb = pool_proxy<64>(kb, Pb);
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) {
            const uint32_t oa = xor_lanes(xa, j), ob = xor_lanes(xb, j);
            const bool keep_min = (size == 64 || (lane & size) == 0) == ((lane & j) == 0);
            xa = keep_min ? min(xa, oa) : max(xa, oa);
            xb = keep_min ? min(xb, ob) : max(xb, ob);
        }
    }
    pool_unproxy<64>(xa, Pa, ka, ia);
    pool_unproxy<64>(xb, Pb, kb, ib);
    pool_finish<64>(v, ua, ka, ia, pa);
    pool_finish<64>(v, ub, kb, ib, pb);
}

// Pool size of owner u (0: past N, its dataset has finished, or it is not an
// owner of the current block of a block-asynchronous iteration: then it
// samples nothing, flips nothing and joins nothing).
__device__ __forceinline__ int pool_size(const Views& v, int u) {
    if (u >= v.N || (v.ds && !pos_active(v, u))) return 0;
    if (v.blk_on && (v.orig[u] < v.blk_lo || v.orig[u] >= v.blk_hi)) return 0;   // not this block's owner
    return v.K + (int)(v.roff[u + 1] - v.roff[u]);
}

// pool_size with the reverse offsets roff[u], roff[u + 1] already read
__device__ __forceinline__ int pool_size_from(const Views& v, int u, uint32_t r0, uint32_t r1) {
    if (u >= v.N || (v.ds && !pos_active(v, u))) return 0;
    if (v.blk_on && (v.orig[u] < v.blk_lo || v.orig[u] >= v.blk_hi)) return 0;   // not this block's owner
    return v.K + (int)(r1 - r0);
}

// Owners in pairs: two pools of at most 32 entries share one wave (one
// 32-lane segment each: a 15-stage sort instead of 21); two pools of at most
// 64 are sorted side by side in the wave's registers; otherwise each owner
// takes the wave alone. Pools of more than 64 entries take the threshold
// select in the same wave when 2C <= 60 (their latency hides behind the
// small pools), else k_select_large (big[u] = 1). Six waves per SIMD: at
// eight (64 VGPRs) the two interleaved pools spill to scratch.
__global__ __launch_bounds__(256, 6) void k_select_small(Views v, uint64_t st0, int t) {
    if (stopped(v)) return;
    __shared__ uint64_t s_key[kSelWaves][64];
    __shared__ uint32_t s_idx[kSelWaves][64];
    __shared__ uint32_t s_cwt[kSelWaves][kThrCache];
    __shared__ uint8_t s_cold[kSelWaves][kThrCache];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int N = v.N;
    const bool thr_inline = 2 * v.C <= 60;
    const int pairs = (N + 1) >> 1;
    // the next pair's reverse offsets are read while this pair is selected
    const int step = gridDim.x * kSelWaves;
    int pr = blockIdx.x * kSelWaves + w;
    uint32_t q0 = 0, q1 = 0, q2 = 0;
    if (pr < pairs) {
        q0 = v.roff[2 * pr];
        q1 = v.roff[2 * pr + 1];
        q2 = v.roff[min(2 * pr + 2, N)];
    }
    for (; pr < pairs; pr += step) {
        const int u0 = 2 * pr, u1 = u0 + 1;
        const uint32_t r0 = q0, r1 = q1, r2 = q2;
        if (pr + step < pairs) {
            q0 = v.roff[2 * (pr + step)];
            q1 = v.roff[2 * (pr + step) + 1];
            q2 = v.roff[min(2 * (pr + step) + 2, N)];
        }
        const int P0 = pool_size_from(v, u0, r0, r1), P1 = pool_size_from(v, u1, r1, r2);
        if (lane == 0) {
            v.big[u0] = P0 > 64 && !thr_inline ? 1u : 0u;
            if (u1 < N) v.big[u1] = P1 > 64 && !thr_inline ? 1u : 0u;
        }
        if (P0 <= 32 && P1 <= 32) {
            const bool hi = lane >= 32;
            select_pool<32>(v, st0, t, hi ? u1 : u0, hi ? P1 : P0);
            continue;
        }
        if (P0 <= 64 && P1 <= 64) {
            select_pool_x2(v, st0, t, u0, P0, u1 < N ? u1 : N, P1);
            continue;
        }
        for (int h = 0; h < 2; ++h) {
            const int u = h ? u1 : u0, P = h ? P1 : P0;
            if (u >= N) break;
            if (P > 64) {
                if (thr_inline)
                    select_large_thr_owner(v, sample_state(v, u, st0, t), u, v.roff[u], P, (uint32_t)v.orig[u],
                                           s_key[w], s_idx[w], s_cwt[w], s_cold[w]);
                continue;
            }
            select_pool<64>(v, st0, t, u, P);
        }
    }
}

void launch_select(const Views& v, uint64_t st, int t, hipStream_t s) {
    hipLaunchKernelGGL(k_select_small, dim3(grid_for((v.N + 1) / 2, kSelWaves, pass_cap(v))), dim3(256), 0, s, v, st, t);
    // The threshold search (inside k_select_small) needs a count in [2C, 64];
    // a member reached by both routes adds two entries of one weight, so the
    // count can step over a window narrower than 3 (2C = 64 leaves one
    // value). Caps above 30 take the rank path.
    if (2 * v.C > 60)
        hipLaunchKernelGGL(k_select_large, dim3(grid_for(v.N, kSelWaves, 4096)), dim3(256), 0, s, v, st, t);
}

// ------------------------------------------------------------------ join (a3, a4)

// Proposals of one owner are bucketed in three steps so that the global
// atomics are one per (owner, target member) instead of one per proposal:
// count per member in LDS, reserve the member's share of its target's bucket
// with one atomicAdd, then write each proposal at base + LDS cursor. The
// capacity of each bucket bounds its proposals by construction; the check
// keeps a violated bound from writing outside it.
struct EmitLds {
    uint32_t* cnt;   // [m] proposals per member (then the cursor)
    uint32_t* base;  // [m] first slot reserved in the member's bucket
    uint32_t* end;   // [m] end of the member's bucket
};

__device__ __forceinline__ void emit_count(const EmitLds& e, int t) { atomicAdd(&e.cnt[t], 1u); }

__device__ __forceinline__ void emit_reserve(const Views& v, const EmitLds& e, const uint32_t* mpos, int m) {
    wave_sync();
    for (int t = lane_id(); t < m; t += 64) {
        const uint32_t c = e.cnt[t];
        const uint32_t pt = mpos[t];
        e.base[t] = c ? bucket_lo(v, (int)pt) + atomicAdd(&v.pcnt[pt], c) : 0u;
        e.end[t] = bucket_lo(v, (int)pt + 1);
        e.cnt[t] = 0u;
    }
    wave_sync();
}

// A proposal is its key alone: the merge finds the source position from the
// id in the key (only for the few ids that enter a list).
__device__ __forceinline__ void emit_write(const Views& v, const EmitLds& e, int t, uint64_t key) {
    const uint32_t slot = e.base[t] + atomicAdd(&e.cnt[t], 1u);
    if (slot < e.end[t]) {
        v.pkey[slot] = key;
    } else {
        atomicOr((unsigned long long*)&v.counters[kCntError], 2ull);
    }
}

__device__ __forceinline__ void emit_clear(const EmitLds& e, int m) {
    for (int t = lane_id(); t < m; t += 64) e.cnt[t] = 0u;
    wave_sync();
}

constexpr int kJoinWaves = 4;

__host__ __device__ static inline size_t join_valu_wave_bytes(const Views& v) {
    const size_t m = 2 * (size_t)v.C;
    return m * v.dp * 4 + m * 28;
}

bool join_valu_fits(const Views& v) { return join_valu_wave_bytes(v) * kJoinWaves <= 64 * 1024; }

// Low-d local join: one wave per owner; member rows staged in LDS, one lane
// per (new member, member) cell; direct-form distances; each pair proposes
// both ways, filtered against the targets' snapshot K-th keys (a proposal not
// below that key can never enter the list). The cells are walked twice:
// once to count proposals per member, once (recomputing the cheap low-d
// distance) to write them.
__global__ __launch_bounds__(256) void k_join_valu(Views v) {
    if (stopped(v)) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int C2 = 2 * v.C, dp = v.dp, dp4 = dp >> 2;
    const double rdp4 = 1.0 / dp4;
    unsigned char* base = smem + (size_t)w * join_valu_wave_bytes(v);
    float* rows = reinterpret_cast<float*>(base);
    uint64_t* thr = reinterpret_cast<uint64_t*>(base + (size_t)C2 * dp * 4);
    uint32_t* oid = reinterpret_cast<uint32_t*>(thr + C2);
    uint32_t* opos = oid + C2;
    EmitLds el{opos + C2, opos + 2 * C2, opos + 3 * C2};
    emit_clear(el, C2);
    const XcdRange xr = xcd_range(v.N, kJoinWaves, w);
    for (int u = xr.next; u < xr.end; u += xr.step) {
        const uint32_t nn = v.nn[u];
        const int nnew = (int)(nn & 0xffffu), m = nnew + (int)(nn >> 16);
        if (nnew == 0) continue;
        if (m > C2) {   // not a sampled neighbourhood: reported, never read
            if (lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 256ull);
            continue;
        }
        const uint2* cs = v.cand + (size_t)u * C2;
        if (v.rk) {   // rows of 4 floats: the row and the K-th key from one record
            for (int i = lane; i < m; i += 64) {
                const uint2 c = cs[i];
                const RowKey* rec = v.rk + c.y;
                const float4 x = rec->x;
                oid[i] = c.x;
                opos[i] = c.y;
                thr[i] = rec->kth;
                reinterpret_cast<float4*>(rows)[i] = x;
            }
            wave_sync();
        } else {
            for (int i = lane; i < m; i += 64) {
                const uint2 c = cs[i];
                oid[i] = c.x;
                opos[i] = c.y;
                thr[i] = v.kth[c.y];
            }
            wave_sync();
            for (int idx = lane; idx < m * dp4; idx += 64) {
                const int r = (int)udiv((uint32_t)idx, (uint32_t)dp4, rdp4), c = idx - r * dp4;
                reinterpret_cast<float4*>(rows)[idx] =
                    reinterpret_cast<const float4*>(v.Xp + (size_t)opos[r] * dp)[c];
            }
            wave_sync();
        }
        const int ncell = nnew * m;
        const double rm = 1.0 / m;
        for (int pass = 0; pass < 2; ++pass) {
            for (int idx = lane; idx < ncell; idx += 64) {
                const int i = (int)udiv((uint32_t)idx, (uint32_t)m, rm), j = idx - i * m;
                if (j < nnew && j <= i) continue;
                const float D = dist_direct(rows + (size_t)i * dp, rows + (size_t)j * dp, dp);
                const uint64_t kb = (uint64_t)__float_as_uint(D) << 32;
                const uint64_t ki = kb | oid[j], kj = kb | oid[i];
                if (pass == 0) {
                    if (ki < thr[i]) emit_count(el, i);
                    if (kj < thr[j]) emit_count(el, j);
                } else {
                    if (ki < thr[i]) emit_write(v, el, i, ki);
                    if (kj < thr[j]) emit_write(v, el, j, kj);
                }
            }
            if (pass == 0) emit_reserve(v, el, opos, m);
        }
        wave_sync();
        emit_clear(el, m);
    }
}

void launch_join_valu(const Views& v, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const size_t lds = join_valu_wave_bytes(v) * kJoinWaves;
    launch_timed(k_join_valu, dim3(grid_for(v.N, kJoinWaves, pass_cap(v))), dim3(256), lds, s, e0, e1, v);
}

// High-d local join on FP32 MFMA (v_mfma_f32_16x16x4f32): per owner, the
// Gram tiles G = A B^T with B = [new | old] member rows and A = the new rows
// (tile rt of A is tile rt of B), only tiles (rt <= ct). Rows are read with
// 32-byte loads per lane: lane (c = lane%16, g = lane/16) holds dims
// [k0 + 8g, k0 + 8g + 8) of member 16*tile + c and feeds component q to
// instruction q. D = ||a||^2 + ||b||^2 - 2 a.b, clamped at 0.
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaMaxCT = 4;   // m = 2C <= 64

// Acc: as in the split form, partial dot products of 16 dimensions (four
// instructions from zero) are added to FP64 accumulators and the distance is
// formed in FP64.
template <bool Acc>
__global__ __launch_bounds__(256) void k_join_mfma(Views v) {
    if (stopped(v)) return;
    __shared__ uint64_t s_thr[kJoinWaves][64];
    __shared__ uint32_t s_oid[kJoinWaves][64];
    __shared__ uint32_t s_pos[kJoinWaves][64];
    __shared__ float s_nrm[kJoinWaves][64];
    __shared__ double s_n64[kJoinWaves][Acc ? 64 : 1];
    __shared__ uint32_t s_emit[kJoinWaves][3][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int C2 = 2 * v.C, dp = v.dp;
    const int c16 = lane & 15, g = lane >> 4;
    EmitLds el{s_emit[w][0], s_emit[w][1], s_emit[w][2]};
    emit_clear(el, 64);
    const XcdRange xr = xcd_range(v.N, kJoinWaves, w);
    for (int u = xr.next; u < xr.end; u += xr.step) {
        const uint32_t nn = v.nn[u];
        const int nnew = (int)(nn & 0xffffu), m = nnew + (int)(nn >> 16);
        if (nnew == 0) continue;
        if (m > C2) {   // not a sampled neighbourhood: reported, never read
            if (lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 256ull);
            continue;
        }
        const uint2* cs = v.cand + (size_t)u * C2;
        if (lane < m) {
            const uint2 c = cs[lane];
            s_oid[w][lane] = c.x;
            s_pos[w][lane] = c.y;
            s_thr[w][lane] = v.kth[c.y];
            if constexpr (Acc)
                s_n64[w][lane] = v.nrm64[c.y];
            else
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
        constexpr int kTiles = kMfmaMaxCT * (kMfmaMaxCT + 1) / 2;
        floatx4 acc[kTiles];
        double a64[Acc ? kTiles : 1][4];
#pragma unroll
        for (int t = 0; t < kTiles; ++t) {
            acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
            if constexpr (Acc)
#pragma unroll
                for (int r = 0; r < 4; ++r) a64[t][r] = 0.0;
        }
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
                if constexpr (Acc) {
                    if (q == 3 || q == 7) {
                        int t2 = 0;
#pragma unroll
                        for (int rt = 0; rt < kMfmaMaxCT; ++rt)
#pragma unroll
                            for (int ct = rt; ct < kMfmaMaxCT; ++ct, ++t2) {
                                if (!(rt < RT && ct < CT)) continue;
#pragma unroll
                                for (int r = 0; r < 4; ++r) a64[t2][r] += (double)acc[t2][r];
                                acc[t2] = floatx4{0.f, 0.f, 0.f, 0.f};
                            }
                    }
                }
            }
        }
        // epilogue: lane holds rows 16rt + 4g + r, column 16ct + c16 of tile t;
        // walked twice (count, then write)
        for (int pass = 0; pass < 2; ++pass) {
            int t = 0;
#pragma unroll
            for (int rt = 0; rt < kMfmaMaxCT; ++rt)
#pragma unroll
                for (int ct = rt; ct < kMfmaMaxCT; ++ct, ++t) {
                    if (!(rt < RT && ct < CT)) continue;
                    const int j = ct * 16 + c16;
                    if (j >= m) continue;
                    const uint32_t oj = s_oid[w][j];
                    const uint64_t tj = s_thr[w][j];
                    const float nj = Acc ? 0.f : s_nrm[w][j];
                    const double nj64 = Acc ? s_n64[w][j] : 0.0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = rt * 16 + g * 4 + r;
                        if (i >= nnew || (j < nnew && j <= i)) continue;
                        float D;
                        if constexpr (Acc)
                            D = (float)((s_n64[w][i] + nj64) - 2.0 * a64[t][r]);
                        else
                            D = (s_nrm[w][i] + nj) - 2.0f * acc[t][r];
                        D = D > 0.f ? D : 0.f;
                        const uint64_t kb = (uint64_t)__float_as_uint(D) << 32;
                        const uint64_t ki = kb | oj, kj = kb | s_oid[w][i];
                        if (pass == 0) {
                            if (ki < s_thr[w][i]) emit_count(el, i);
                            if (kj < tj) emit_count(el, j);
                        } else {
                            if (ki < s_thr[w][i]) emit_write(v, el, i, ki);
                            if (kj < tj) emit_write(v, el, j, kj);
                        }
                    }
                }
            if (pass == 0) emit_reserve(v, el, s_pos[w], m);
        }
        wave_sync();
        emit_clear(el, m);
    }
}

void launch_join_mfma(const Views& v, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 g(grid_for(v.N, kJoinWaves, pass_cap(v)));
    if (v.acc)
        launch_timed(k_join_mfma<true>, g, dim3(256), 0, s, e0, e1, v);
    else
        launch_timed(k_join_mfma<false>, g, dim3(256), 0, s, e0, e1, v);
}

// ------------------------------------------------------------------ precision form (a9)
//
// BF16 copies of the rows feed BF16 MFMA Gram tiles with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16) as a screen; every direction that can pass the
// snapshot filter is rescored in FP32 from the original rows, and only the
// rescored distances are proposed, filtered exactly and stored.
//
// Screen bound. With x~ = bf16(x) and e_x = ||x~ - x|| (the row's rounding
// error, computed exactly when the copies are made: x~_j - x_j is exact in
// FP32, its squares and sum are taken in FP64; e_x = 0 for rows exact in
// BF16, such as 8-bit pixels, and e_x <= 2^-8 ||x|| always),
// | ||x~-y~|| - ||x-y|| | <= ||(x~-x) - (y~-y)|| <= eps = e_x + e_y, so
// |D~e - D| <= 2 eps sqrt(D) + eps^2 for D~e the exact distance of the BF16
// rows. The tile computes D~ = n~x + n~y - 2 x~.y~ in FP32 (BF16 products are
// exact in FP32) with |D~ - D~e| <= (d+3) 2^-24 (||x~|| + ||y~||)^2. A pair with
// D <= T therefore has D~ <= T + 2 eps sqrt(T) + eps^2 + (d+3) 2^-24
// (||x~|| + ||y~||)^2, the test applied (in FP64, with the bound enlarged by
// 2^-20 relative).
//
// Rescore. The owner's member rows (FP32, the original values) are staged in
// LDS 32 dimensions at a time, so each member row is read once per owner, as
// the join reads it; one lane per surviving pair adds the chunk's squared
// differences into four partial sums (components 0..3 of its eight 16-byte
// groups, in dimension order), adds (s0 + s1) + (s2 + s3) to an FP64 total in
// chunk order, and rounds the total to FP32 once. The value depends on the
// two rows alone, and swapping them only negates the differences: one key per
// pair whichever owner evaluates it, deterministic.
// Error (u = 2^-24, terms non-negative): a term (x_j - y_j)^2 carries at most
// 2u, eight accumulations and two adds at most 10u more, the FP64 total and
// its rounding at most 0.5u + d 2^-53, so |D' - D| <= 13u D at any d. The
// screen adds 16u T to its margin, so that no pair whose rescored key passes
// the filter is screened out.

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__global__ void k_make_bf16(Views v) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < v.N; p += gridDim.x * blockDim.x) {
        const float* x = v.Xp + (size_t)p * v.dp;
        uint16_t* y = v.Xb + (size_t)p * v.dp;
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
        double r = 0.0;   // sum of squared rounding errors (each exact in FP32, squares exact in FP64)
        for (int j = 0; j < v.dp; j += 4) {
            const float4 a = *reinterpret_cast<const float4*>(x + j);
            const uint16_t b0 = bf16_rne(a.x), b1 = bf16_rne(a.y), b2 = bf16_rne(a.z), b3 = bf16_rne(a.w);
            y[j] = b0;
            y[j + 1] = b1;
            y[j + 2] = b2;
            y[j + 3] = b3;
            const float f0 = bf16_to_f32(b0), f1 = bf16_to_f32(b1), f2 = bf16_to_f32(b2), f3 = bf16_to_f32(b3);
            s0 = fmaf(f0, f0, s0);
            s1 = fmaf(f1, f1, s1);
            s2 = fmaf(f2, f2, s2);
            s3 = fmaf(f3, f3, s3);
            const double e0 = (double)(f0 - a.x), e1 = (double)(f1 - a.y), e2 = (double)(f2 - a.z),
                         e3 = (double)(f3 - a.w);
            r += (e0 * e0 + e1 * e1) + (e2 * e2 + e3 * e3);
        }
        // the FP64 sum's relative error (below d 2^-53) and the FP32 rounding of
        // the norm (2^-24) are covered by the 2^-20 enlargement of the bound
        v.nb[p] = make_float2((s0 + s1) + (s2 + s3), (float)(sqrt(r) * (1.0 + 1.0 / 1073741824.0)));
    }
}

void launch_make_bf16(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_make_bf16, dim3(grid_for(v.N, 256, 8192)), dim3(256), 0, s, v);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kRsChunk = 32;             // dimensions staged per pass (dp % 32 == 0 on this path)
constexpr int kRsStride = kRsChunk + 4;  // floats per staged row: the 16-byte pad spreads rows over the banks

// Most pairs one owner evaluates (new x new unordered, new x old): the bound
// on its survivors.
__host__ __device__ inline int bf_max_surv(int C) { return C * (C - 1) / 2 + C * C; }

// Per-wave dynamic LDS of the precision-form join: staged rows [2C][kRsStride]
// floats, FP64 rescore totals [S], survivors [S] as uint16.
__host__ __device__ inline size_t bf_rows_bytes(int C) { return (size_t)2 * C * kRsStride * 4; }
__host__ __device__ inline size_t bf_wave_bytes(int C) {
    const size_t S = (size_t)bf_max_surv(C);
    return bf_rows_bytes(C) + S * 8 + ((S * 2 + 15) & ~(size_t)15);
}

typedef float floatx32 __attribute__((ext_vector_type(32)));

// Rescore of one owner's survivors. Lane l stages 16 bytes of rows
// l/8 + 8k (k < NG = ceil(m/8); rows past m repeat row m-1 in the loads and
// are not stored). Two register buffers alternate over the chunks, so the
// loads of the next two chunks are in flight while one is summed; the staged
// values sit in vector register tuples (element 4k + c), which stay in
// registers at any NG. Survivor q (i | j << 6 | directions << 12) is summed
// by lane q mod 64 into s_tot[q].
template <int NG>
__device__ __forceinline__ void stage_load(floatx32& buf, const float* const (&src)[NG], int off) {
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        const float4 x = *reinterpret_cast<const float4*>(src[k] + off);
        buf[4 * k] = x.x;
        buf[4 * k + 1] = x.y;
        buf[4 * k + 2] = x.z;
        buf[4 * k + 3] = x.w;
    }
}

template <int NG>
__device__ __forceinline__ void stage_store(const floatx32& buf, float* s_rows, int sr, int sc, int m) {
#pragma unroll
    for (int k = 0; k < NG; ++k)
        if (sr + 8 * k < m)
            *reinterpret_cast<float4*>(s_rows + (sr + 8 * k) * kRsStride + sc) =
                make_float4(buf[4 * k], buf[4 * k + 1], buf[4 * k + 2], buf[4 * k + 3]);
    wave_sync();
}

__device__ __forceinline__ void rescore_chunk(const uint16_t* s_surv, double* s_tot, uint32_t nsv,
                                              const float* s_rows) {
    for (uint32_t q = (uint32_t)lane_id(); q < nsv; q += 64) {
        const uint32_t e = s_surv[q];
        const float4* pa = reinterpret_cast<const float4*>(s_rows + (e & 63u) * kRsStride);
        const float4* pb = reinterpret_cast<const float4*>(s_rows + ((e >> 6) & 63u) * kRsStride);
        s_tot[q] += (double)chunk32_sq(pa, pb);
    }
    wave_sync();
}

template <int NG>
__device__ __forceinline__ void rescore_staged(const Views& v, const uint32_t* pos, int m, const uint16_t* s_surv,
                                               double* s_tot, uint32_t nsv, float* s_rows) {
    const int lane = lane_id(), dp = v.dp;
    const int sr = lane >> 3, sc = (lane & 7) * 4;
    const float* src[NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) src[k] = v.Xp + (size_t)pos[min(sr + 8 * k, m - 1)] * dp + sc;
    // straight-line loads (the last chunks are loaded again past the end),
    // so that only the loads of the chunk being stored are waited for
    const int last = dp - kRsChunk;
    floatx32 A, B;
    stage_load<NG>(A, src, 0);
    stage_load<NG>(B, src, min(kRsChunk, last));
    for (uint32_t q = (uint32_t)lane; q < nsv; q += 64) s_tot[q] = 0.0;
    for (int k0 = 0; k0 < dp; k0 += 2 * kRsChunk) {
        stage_store<NG>(A, s_rows, sr, sc, m);
        stage_load<NG>(A, src, min(k0 + 2 * kRsChunk, last));
        rescore_chunk(s_surv, s_tot, nsv, s_rows);
        const bool odd = k0 + kRsChunk < dp;
        if (odd) stage_store<NG>(B, s_rows, sr, sc, m);
        stage_load<NG>(B, src, min(k0 + 3 * kRsChunk, last));
        if (odd) rescore_chunk(s_surv, s_tot, nsv, s_rows);
    }
}

// MaxCT column tiles of 16 members (2C <= 16 MaxCT); NGmax = ceil(2C / 8)
// row groups staged per lane in the rescore: both follow the sample cap, so
// the register budget (and the waves resident) does too.
template <int MaxCT, int NGmax>
__global__ __launch_bounds__(256, MaxCT <= 2 ? 3 : 2) void k_join_bf16(Views v) {
    if (stopped(v)) return;
    __shared__ uint64_t s_thr[kJoinWaves][64];
    __shared__ uint32_t s_oid[kJoinWaves][64];
    __shared__ uint32_t s_pos[kJoinWaves][64];
    __shared__ float s_nb[kJoinWaves][64];
    __shared__ float s_eb[kJoinWaves][64];   // rounding-error norm of the member's BF16 row
    __shared__ double s_sn[kJoinWaves][64];  // sqrt of the BF16 squared norm
    __shared__ double s_st[kJoinWaves][64];  // sqrt of the snapshot threshold distance
    __shared__ uint32_t s_emit[kJoinWaves][3][64];
    extern __shared__ __align__(16) unsigned char s_dyn[];
    const int lane = lane_id(), w = threadIdx.x >> 6, wpb = (int)(blockDim.x >> 6);
    const int C2 = 2 * v.C, dp = v.dp;
    const int S = bf_max_surv(v.C);
    unsigned char* wbase = s_dyn + (size_t)w * bf_wave_bytes(v.C);
    float* s_rows = reinterpret_cast<float*>(wbase);
    double* s_tot = reinterpret_cast<double*>(wbase + bf_rows_bytes(v.C));
    uint16_t* s_surv = reinterpret_cast<uint16_t*>(wbase + bf_rows_bytes(v.C) + (size_t)S * 8);
    const int c16 = lane & 15, g = lane >> 4;
    EmitLds el{s_emit[w][0], s_emit[w][1], s_emit[w][2]};
    emit_clear(el, 64);
    uint64_t rescored = 0;
    const double cfp = (double)(dp + 3) * (1.0 / 16777216.0);
    const double crs = 16.0 / 16777216.0;   // the rescore's relative error (at most 13u), with room
    const XcdRange xr = xcd_range(v.N, wpb, w);
    for (int u = xr.next; u < xr.end; u += xr.step) {
        const uint32_t nn = v.nn[u];
        const int nnew = (int)(nn & 0xffffu), m = nnew + (int)(nn >> 16);
        if (nnew == 0) continue;
        if (m > C2) {   // not a sampled neighbourhood: reported, never read
            if (lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 256ull);
            continue;
        }
        const uint2* cs = v.cand + (size_t)u * C2;
        if (lane < m) {
            const uint2 c = cs[lane];
            s_oid[w][lane] = c.x;
            s_pos[w][lane] = c.y;
            const uint64_t thr = v.kth[c.y];
            const float2 nb = v.nb[c.y];
            s_thr[w][lane] = thr;
            s_nb[w][lane] = nb.x;
            s_eb[w][lane] = nb.y;
            s_sn[w][lane] = sqrt((double)nb.x);
            s_st[w][lane] = sqrt((double)__uint_as_float((uint32_t)(thr >> 32)));
        }
        wave_sync();
        const int RT = (nnew + 15) >> 4, CT = (m + 15) >> 4;
        const uint16_t* rp[MaxCT];
        bool rv[MaxCT];
        for (int ct = 0; ct < MaxCT; ++ct) {
            const int j = ct * 16 + c16;
            rv[ct] = ct < CT && j < m;
            rp[ct] = v.Xb + (size_t)(rv[ct] ? s_pos[w][j] : 0u) * dp + g * 8;
        }
        floatx4 acc[MaxCT * (MaxCT + 1) / 2];
        for (int t = 0; t < MaxCT * (MaxCT + 1) / 2; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < dp; k0 += 32) {
            bf16x8 f[MaxCT];
#pragma unroll
            for (int ct = 0; ct < MaxCT; ++ct) {
                uint4 raw = make_uint4(0u, 0u, 0u, 0u);
                if (rv[ct]) raw = *reinterpret_cast<const uint4*>(rp[ct] + k0);
                f[ct] = __builtin_bit_cast(bf16x8, raw);
            }
            int t = 0;
#pragma unroll
            for (int rt = 0; rt < MaxCT; ++rt)
#pragma unroll
                for (int ct = rt; ct < MaxCT; ++ct, ++t)
                    if (rt < RT && ct < CT)
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[rt], f[ct], acc[t], 0, 0, 0);
        }
        // screen: every cell and direction that can pass the snapshot filter
        uint32_t nsv = 0;
        {
            int t = 0;
#pragma unroll
            for (int rt = 0; rt < MaxCT; ++rt)
#pragma unroll
                for (int ct = rt; ct < MaxCT; ++ct, ++t) {
                    if (!(rt < RT && ct < CT)) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = rt * 16 + g * 4 + r, j = ct * 16 + c16;
                        bool si = false, sj = false;
                        if (j < m && i < nnew && !(j < nnew && j <= i)) {
                            const double Dt = (double)((s_nb[w][i] + s_nb[w][j]) - 2.0f * acc[t][r]);
                            const double eps = (double)s_eb[w][i] + (double)s_eb[w][j];
                            const double nbs = s_sn[w][i] + s_sn[w][j];
                            const double fp = cfp * nbs * nbs;
                            const double Ti = (double)__uint_as_float((uint32_t)(s_thr[w][i] >> 32));
                            const double Tj = (double)__uint_as_float((uint32_t)(s_thr[w][j] >> 32));
                            const double mi =
                                (2.0 * eps * s_st[w][i] + eps * eps + fp) * (1.0 + 1.0 / 1048576.0) + crs * Ti;
                            const double mj =
                                (2.0 * eps * s_st[w][j] + eps * eps + fp) * (1.0 + 1.0 / 1048576.0) + crs * Tj;
                            si = Dt - mi <= Ti;
                            sj = Dt - mj <= Tj;
                        }
                        const bool sv = si || sj;
                        const uint64_t mk = ballot(sv);
                        const uint32_t slot = nsv + mbcnt(mk);
                        if (sv && slot < (uint32_t)S)
                            s_surv[slot] = (uint16_t)((uint32_t)i | ((uint32_t)j << 6) | (si ? 1u << 12 : 0u) |
                                                      (sj ? 1u << 13 : 0u));
                        nsv += (uint32_t)__popcll(mk);
                    }
                }
        }
        if (nsv > (uint32_t)S) {  // cannot happen: survivors <= e(u) <= S
            if (lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 128ull);
            nsv = (uint32_t)S;
        }
        wave_sync();
        // rescore from the FP32 rows staged 32 dimensions at a time
        switch (min(__builtin_amdgcn_readfirstlane((m + 7) >> 3), NGmax)) {
            case 1: rescore_staged<1>(v, s_pos[w], m, s_surv, s_tot, nsv, s_rows); break;
            case 2: rescore_staged<(NGmax < 2 ? NGmax : 2)>(v, s_pos[w], m, s_surv, s_tot, nsv, s_rows); break;
            case 3: rescore_staged<(NGmax < 3 ? NGmax : 3)>(v, s_pos[w], m, s_surv, s_tot, nsv, s_rows); break;
            case 4: rescore_staged<(NGmax < 4 ? NGmax : 4)>(v, s_pos[w], m, s_surv, s_tot, nsv, s_rows); break;
            case 5: rescore_staged<(NGmax < 5 ? NGmax : 5)>(v, s_pos[w], m, s_surv, s_tot, nsv, s_rows); break;
            case 6: rescore_staged<(NGmax < 6 ? NGmax : 6)>(v, s_pos[w], m, s_surv, s_tot, nsv, s_rows); break;
            case 7: rescore_staged<(NGmax < 7 ? NGmax : 7)>(v, s_pos[w], m, s_surv, s_tot, nsv, s_rows); break;
            default: rescore_staged<NGmax>(v, s_pos[w], m, s_surv, s_tot, nsv, s_rows); break;
        }
        rescored += nsv;
        // exact filter on the rescored keys: count, reserve, write
        for (int pass = 0; pass < 2; ++pass) {
            for (uint32_t q = (uint32_t)lane; q < nsv; q += 64) {
                const uint32_t e = s_surv[q];
                const int a = (int)(e & 63u), b = (int)((e >> 6) & 63u);
                const uint64_t kb = (uint64_t)__float_as_uint((float)s_tot[q]) << 32;
                const uint64_t ka = kb | s_oid[w][b], kbb = kb | s_oid[w][a];
                const bool da = (e >> 12) & 1u, db = (e >> 13) & 1u;
                if (pass == 0) {
                    if (da && ka < s_thr[w][a]) emit_count(el, a);
                    if (db && kbb < s_thr[w][b]) emit_count(el, b);
                } else {
                    if (da && ka < s_thr[w][a]) emit_write(v, el, a, ka);
                    if (db && kbb < s_thr[w][b]) emit_write(v, el, b, kbb);
                }
            }
            if (pass == 0) emit_reserve(v, el, s_pos[w], m);
        }
        wave_sync();
        emit_clear(el, m);
    }
    if (lane == 0 && rescored) atomicAdd((unsigned long long*)&v.counters[kCntRescored], (unsigned long long)rescored);
}

// Waves per workgroup: four where the device's LDS per workgroup holds them.
template <int MaxCT, int NGmax>
static void launch_bf16(const Views& v, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    static const int lds_max = [] {
        int dev = 0, lim = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lim <= 0)
            lim = 65536;
        return lim;
    }();
    static const size_t lds_static = [] {
        hipFuncAttributes a{};
        return hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_join_bf16<MaxCT, NGmax>)) == hipSuccess
                   ? (size_t)a.sharedSizeBytes
                   : (size_t)kJoinWaves * 64 * 52;
    }();
    const size_t wb = bf_wave_bytes(v.C);
    int wpb = kJoinWaves;
    while (wpb > 1 && lds_static + (size_t)wpb * wb > (size_t)lds_max) wpb >>= 1;
    const size_t lds = (size_t)wpb * wb;
    if (lds > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_join_bf16<MaxCT, NGmax>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    launch_timed(k_join_bf16<MaxCT, NGmax>, dim3(grid_for(v.N, wpb, pass_cap(v))), dim3(64 * wpb), lds, s, e0, e1,
                 v);
}

void launch_join_bf16(const Views& v, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int C2 = 2 * v.C;
    if (C2 <= 24)
        launch_bf16<2, 3>(v, s, e0, e1);
    else if (C2 <= 32)
        launch_bf16<2, 4>(v, s, e0, e1);
    else if (C2 <= 40)
        launch_bf16<3, 5>(v, s, e0, e1);
    else if (C2 <= 48)
        launch_bf16<3, 6>(v, s, e0, e1);
    else
        launch_bf16<4, 8>(v, s, e0, e1);
}

// ------------------------------------------------------------------ split-BF16 Gram form
//
// x = x1 + x2 + x3 exactly: x1 = bf16(x) (round to nearest even), r1 = x - x1
// is exact in FP32 and has at most 16 significant bits, x2 = bf16(r1), and
// r1 - x2 has at most 8 significant bits, so x3 = bf16(r1 - x2) = r1 - x2.
// x.y = sum_{i,j} xi yj; the tiles accumulate the six products with i + j <= 4
// (BF16 x BF16 is exact in FP32). The dropped x2y3 + x3y2 + x3y3 is below
// 2^-25 |x_k y_k| per term (|x2| <= 2^-9 |x|, |x3| <= 2^-17 |x|).
//
// Symmetry. A pair is evaluated by several owners, as row or as column, and
// the merge needs one key per pair. Three accumulators per tile, each taking
// its two products in a fixed order per 32-dimension step:
//   S = x2.y2 then x1.y1,   R = x1.y3 then x1.y2,   Q = x3.y1 then x2.y1.
// Swapping the roles of x and y leaves S unchanged and exchanges R and Q
// (the same products in the same order), so x.y = S + (R + Q) is the same
// FP32 value either way.

// Also records which planes hold a nonzero value (counter kCntSplit; one
// atomic per wave): planes that are all zero contribute exact zeros and the
// join skips them.
__global__ void k_make_split(Views v) {
    const int64_t total = (int64_t)v.N * v.dp;
    uint32_t used = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = v.Xp[i];
        const uint16_t b1 = bf16_rne(x);
        const float r1 = x - bf16_to_f32(b1);
        const uint16_t b2 = bf16_rne(r1);
        const float r2 = r1 - bf16_to_f32(b2);
        const uint16_t b3 = bf16_rne(r2);
        v.Xs[i] = b1;
        v.Xs[total + i] = b2;
        v.Xs[2 * total + i] = b3;
        used |= (b2 ? 1u : 0u) | (b3 ? 2u : 0u);
    }
    const uint64_t m1 = ballot((used & 1u) != 0), m2 = ballot((used & 2u) != 0);
    const uint32_t wu = (m1 ? 1u : 0u) | (m2 ? 2u : 0u);
    if (lane_id() == 0 && wu) flag_or(&v.counters[kCntSplit], wu);
}

void launch_make_split(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_make_split, dim3(grid_for((int64_t)v.N * v.dp, 1024, 16384)), dim3(256), 0, s, v);
}

// Layout of the MFMA forms in one pass over X, one wave per row: the squared
// norm (lane sums over j mod 4, then a fixed xor tree), identity positions,
// the finiteness check, and either the padded FP32 row (FP32 tiles) or, for
// the split form, the first BF16 plane and the used-plane record of
// k_make_split. The FP32 row and planes 2 and 3 of the split form are
// written by k_prep_rest only when a later plane is used (no reader needs
// them otherwise).
__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ X, Views v, int split) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int d = v.d, dp = v.dp;
    bool bad = false;
    uint32_t used = 0;
    for (int r = blockIdx.x * 4 + w; r < v.N; r += gridDim.x * 4) {
        const float* x = X + (size_t)r * d;
        float* y = v.Xp + (size_t)r * dp;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int j = 4 * lane; j < dp; j += 256) {
            float4 q;
            q.x = j < d ? x[j] : 0.f;
            q.y = j + 1 < d ? x[j + 1] : 0.f;
            q.z = j + 2 < d ? x[j + 2] : 0.f;
            q.w = j + 3 < d ? x[j + 3] : 0.f;
            bad |= ((__float_as_uint(q.x) | 0u) & 0x7f800000u) == 0x7f800000u ||
                   (__float_as_uint(q.y) & 0x7f800000u) == 0x7f800000u ||
                   (__float_as_uint(q.z) & 0x7f800000u) == 0x7f800000u ||
                   (__float_as_uint(q.w) & 0x7f800000u) == 0x7f800000u;
            // squares exact in FP64; integrality decides whether FP32 Gram sums are exact
            s0 = fma((double)q.x, (double)q.x, s0);
            s1 = fma((double)q.y, (double)q.y, s1);
            s2 = fma((double)q.z, (double)q.z, s2);
            s3 = fma((double)q.w, (double)q.w, s3);
            if (q.x != rintf(q.x) || q.y != rintf(q.y) || q.z != rintf(q.z) || q.w != rintf(q.w)) used |= 4u;
            if (split) {
                // byte rows (read instead of plane 1 when every value is an integer in 0..255)
                const float e8[4] = {q.x, q.y, q.z, q.w};
                uint32_t packed = 0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const bool in = e8[c] >= 0.f && e8[c] <= 255.f;
                    if (!in) used |= 16u;
                    packed |= (in ? (uint32_t)e8[c] : 0u) << (8 * c);
                }
                *reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(v.Xs + (size_t)v.N * dp) + (size_t)r * dp + j) =
                    packed;
                const float e[4] = {q.x, q.y, q.z, q.w};
                uint16_t b1[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    b1[c] = bf16_rne(e[c]);
                    const float r1 = e[c] - bf16_to_f32(b1[c]);
                    const uint16_t b2 = bf16_rne(r1);
                    const uint16_t b3 = bf16_rne(r1 - bf16_to_f32(b2));
                    used |= (b2 ? 1u : 0u) | (b3 ? 2u : 0u);
                }
                *reinterpret_cast<uint2*>(v.Xs + (size_t)r * dp + j) =
                    make_uint2(b1[0] | ((uint32_t)b1[1] << 16), b1[2] | ((uint32_t)b1[3] << 16));
            } else {
                *reinterpret_cast<float4*>(y + j) = q;
            }
        }
        double sn = (s0 + s1) + (s2 + s3);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sn += __shfl_xor(sn, o);
        if (sn > 8388608.0) used |= 8u;   // above 2^23: n(x) + n(y) may round in FP32
        if (lane == 0) {
            v.nrm64[r] = sn;
            v.nrm[r] = (float)sn;
            v.orig[r] = r;
            v.posof[r] = r;
        }
    }
    const uint64_t m1 = ballot((used & 1u) != 0), m2 = ballot((used & 2u) != 0), mb = ballot(bad);
    const uint64_t m4 = ballot((used & 4u) != 0), m8 = ballot((used & 8u) != 0), m16 = ballot((used & 16u) != 0);
    if (lane == 0) {
        const uint32_t wu = (m1 ? 1u : 0u) | (m2 ? 2u : 0u) | (m4 ? 4u : 0u) | (m8 ? 8u : 0u) | (m16 ? 16u : 0u);
        if (wu) flag_or(&v.counters[kCntSplit], wu);
        if (mb) flag_or(&v.counters[kCntNonFinite], 1ull);
    }
}

void launch_prep(const float* X, const Views& v, int split, hipStream_t s) {
    hipLaunchKernelGGL(k_prep, dim3(grid_for(v.N, 4, 16384)), dim3(256), 0, s, X, v, split);
}

// Split form with a later plane in use: the padded FP32 rows and planes 2
// and 3 (plane 1 is already written by k_prep).
__global__ __launch_bounds__(256) void k_prep_rest(const float* __restrict__ X, Views v) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int d = v.d, dp = v.dp;
    const int64_t total = (int64_t)v.N * dp;
    for (int r = blockIdx.x * 4 + w; r < v.N; r += gridDim.x * 4) {
        const float* x = X + (size_t)r * d;
        float* y = v.Xp + (size_t)r * dp;
        for (int j = 4 * lane; j < dp; j += 256) {
            float4 q;
            q.x = j < d ? x[j] : 0.f;
            q.y = j + 1 < d ? x[j + 1] : 0.f;
            q.z = j + 2 < d ? x[j + 2] : 0.f;
            q.w = j + 3 < d ? x[j + 3] : 0.f;
            *reinterpret_cast<float4*>(y + j) = q;
            const float e[4] = {q.x, q.y, q.z, q.w};
            uint16_t b2[4], b3[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float r1 = e[c] - bf16_to_f32(bf16_rne(e[c]));
                b2[c] = bf16_rne(r1);
                b3[c] = bf16_rne(r1 - bf16_to_f32(b2[c]));
            }
            const size_t at = (size_t)r * dp + j;
            *reinterpret_cast<uint2*>(v.Xs + total + at) =
                make_uint2(b2[0] | ((uint32_t)b2[1] << 16), b2[2] | ((uint32_t)b2[3] << 16));
            *reinterpret_cast<uint2*>(v.Xs + 2 * total + at) =
                make_uint2(b3[0] | ((uint32_t)b3[1] << 16), b3[2] | ((uint32_t)b3[3] << 16));
        }
    }
}

void launch_prep_rest(const float* X, const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_prep_rest, dim3(grid_for(v.N, 4, 16384)), dim3(256), 0, s, X, v);
}

// The tiles of k_join_mfma on BF16 MFMA (v_mfma_f32_16x16x32_bf16): lane
// (c = lane%16, g = lane/16) holds dims [k0 + 8g, k0 + 8g + 8) of member
// 16*tile + c in each of the three planes; A and B take the same lane-to-k
// map. Rows are new members only (nnew <= C <= 32: row tiles 0 and 1).
// Epilogue as in the FP32 kernel.
// MaxCT column tiles (m = 2C <= 16 MaxCT); rows are new members, nnew <= 32,
// so row tiles 0 and 1 only: 2 MaxCT - 1 tiles.
// Acc (data whose FP32 sums are not exact): S, the dominant x1.y1 term,
// restarts at zero every 32-dimension step and each step's S is added to an
// FP64 accumulator; R and Q (cross terms at most 2^-8 of it) accumulate in
// FP32 over all steps as before. x.y = S64 + (R + Q) in FP64 is still the
// same value with x and y exchanged, and the distance is formed from FP64
// norms in FP64 and rounded once.
// U8 (8-bit data, one plane, FP32 sums exact): the rows are read as bytes
// (half the bytes of the BF16 plane) and widened to BF16 in registers, each
// byte exactly; the tiles and their order are those of the plane form, so
// every distance is bit-identical to it.
__device__ __forceinline__ uint32_t u8x2_to_bf16x2(uint32_t w, int k) {
    const uint32_t lo = __float_as_uint((float)((w >> (8 * k)) & 0xffu));
    const uint32_t hi = __float_as_uint((float)((w >> (8 * k + 8)) & 0xffu));
    return (lo >> 16) | (hi & 0xffff0000u);
}

template <int MaxCT, int Planes, bool Acc, bool U8 = false>
__global__ __launch_bounds__(256, U8 ? (MaxCT <= 2 ? 6 : MaxCT <= 3 ? 5 : 3) : MaxCT <= 2 ? ((Acc && Planes == 3) ? 3 : 4) : (MaxCT <= 3 && !(Acc && Planes >= 2)) ? 3 : 2)
void k_join_split(Views v) {
    static_assert(!U8 || (Planes == 1 && !Acc), "byte rows carry one exact plane");
    if (stopped(v)) return;
    constexpr int kSplitTiles = 2 * MaxCT - 1;
    __shared__ uint64_t s_thr[kJoinWaves][64];
    __shared__ uint32_t s_oid[kJoinWaves][64];
    __shared__ uint32_t s_pos[kJoinWaves][64];
    __shared__ float s_nrm[kJoinWaves][64];
    __shared__ double s_n64[kJoinWaves][Acc ? 64 : 1];
    __shared__ uint32_t s_emit[kJoinWaves][3][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int C2 = 2 * v.C, dp = v.dp;
    const size_t plane = (size_t)v.N * dp;
    const int c16 = lane & 15, g = lane >> 4;
    EmitLds el{s_emit[w][0], s_emit[w][1], s_emit[w][2]};
    emit_clear(el, 64);
    const XcdRange xr = xcd_range(v.N, kJoinWaves, w);
    for (int u = xr.next; u < xr.end; u += xr.step) {
        const uint32_t nn = v.nn[u];
        const int nnew = (int)(nn & 0xffffu), m = nnew + (int)(nn >> 16);
        if (nnew == 0) continue;
        if (m > C2) {   // not a sampled neighbourhood: reported, never read
            if (lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 256ull);
            continue;
        }
        const uint2* cs = v.cand + (size_t)u * C2;
        if (lane < m) {
            const uint2 c = cs[lane];
            s_oid[w][lane] = c.x;
            s_pos[w][lane] = c.y;
            s_thr[w][lane] = v.kth[c.y];
            if constexpr (Acc)
                s_n64[w][lane] = v.nrm64[c.y];
            else
                s_nrm[w][lane] = v.nrm[c.y];
        }
        wave_sync();
        const int RT = (nnew + 15) >> 4, CT = (m + 15) >> 4;
        // lanes past the last member read member m-1; their outputs are never used
        const uint16_t* rp[MaxCT];
        const uint8_t* rb[MaxCT];
        const uint8_t* bytes = reinterpret_cast<const uint8_t*>(v.Xs + plane);
#pragma unroll
        for (int ct = 0; ct < MaxCT; ++ct) {
            const size_t row = (size_t)s_pos[w][min(ct * 16 + c16, m - 1)] * dp + g * 8;
            rp[ct] = v.Xs + row;
            rb[ct] = bytes + row;
        }
        floatx4 aS[kSplitTiles], aR[kSplitTiles], aQ[kSplitTiles];
        double a64[Acc ? kSplitTiles : 1][4];
#pragma unroll
        for (int t = 0; t < kSplitTiles; ++t) {
            aS[t] = floatx4{0.f, 0.f, 0.f, 0.f};
            aR[t] = floatx4{0.f, 0.f, 0.f, 0.f};
            aQ[t] = floatx4{0.f, 0.f, 0.f, 0.f};
            if constexpr (Acc)
#pragma unroll
                for (int r = 0; r < 4; ++r) a64[t][r] = 0.0;
        }
        int k0 = 0;
        if constexpr (U8) {
            // 64 dimensions per step: each lane loads 16 bytes (half the load
            // instructions of 8-byte loads) and feeds two instructions; lane
            // (c16, g) takes bytes [k0 + 16 g, k0 + 16 g + 16) of its row for
            // both operands, so every instruction pairs the same dimensions
            // (exact sums: the order of the partial products is free)
            const uint8_t* rw[MaxCT];
#pragma unroll
            for (int ct = 0; ct < MaxCT; ++ct) rw[ct] = rb[ct] + g * 8;
            for (; k0 + 64 <= dp; k0 += 64) {
                bf16x8 lo[MaxCT], hi[MaxCT];
#pragma unroll
                for (int ct = 0; ct < MaxCT; ++ct) {
                    uint4 b16 = make_uint4(0u, 0u, 0u, 0u);
                    if (ct < CT) b16 = *reinterpret_cast<const uint4*>(rw[ct] + k0);
                    lo[ct] = __builtin_bit_cast(bf16x8, make_uint4(u8x2_to_bf16x2(b16.x, 0), u8x2_to_bf16x2(b16.x, 2),
                                                                   u8x2_to_bf16x2(b16.y, 0), u8x2_to_bf16x2(b16.y, 2)));
                    hi[ct] = __builtin_bit_cast(bf16x8, make_uint4(u8x2_to_bf16x2(b16.z, 0), u8x2_to_bf16x2(b16.z, 2),
                                                                   u8x2_to_bf16x2(b16.w, 0), u8x2_to_bf16x2(b16.w, 2)));
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    int t = 0;
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                        for (int ct = rt; ct < MaxCT; ++ct, ++t) {
                            if (!(rt < RT && ct < CT)) continue;
                            aS[t] = h ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[rt], hi[ct], aS[t], 0, 0, 0)
                                      : __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[rt], lo[ct], aS[t], 0, 0, 0);
                        }
                }
            }
        }
        for (; k0 < dp; k0 += 32) {
            bf16x8 f[Planes][MaxCT];
#pragma unroll
            for (int q = 0; q < Planes; ++q)
#pragma unroll
                for (int ct = 0; ct < MaxCT; ++ct) {
                    uint4 raw = make_uint4(0u, 0u, 0u, 0u);
                    if constexpr (U8) {
                        if (ct < CT) {
                            const uint2 b8 = *reinterpret_cast<const uint2*>(rb[ct] + k0);
                            raw = make_uint4(u8x2_to_bf16x2(b8.x, 0), u8x2_to_bf16x2(b8.x, 2), u8x2_to_bf16x2(b8.y, 0),
                                             u8x2_to_bf16x2(b8.y, 2));
                        }
                    } else {
                        if (ct < CT) raw = *reinterpret_cast<const uint4*>(rp[ct] + q * plane + k0);
                    }
                    f[q][ct] = __builtin_bit_cast(bf16x8, raw);
                }
            // product kinds outer, tiles inner: consecutive instructions go to
            // different accumulators
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                int t = 0;
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int ct = rt; ct < MaxCT; ++ct, ++t) {
                        if (!(rt < RT && ct < CT)) continue;
                        // products with an all-zero plane are exact zeros: skipped
                        if constexpr (Planes >= 2) {
                            if (q == 0) aS[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[1][rt], f[1][ct], aS[t], 0, 0, 0);
                            if (q == 4) aR[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[0][rt], f[1][ct], aR[t], 0, 0, 0);
                            if (q == 5) aQ[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[1][rt], f[0][ct], aQ[t], 0, 0, 0);
                        }
                        if constexpr (Planes >= 3) {
                            if (q == 1) aR[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[0][rt], f[2][ct], aR[t], 0, 0, 0);
                            if (q == 2) aQ[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[2][rt], f[0][ct], aQ[t], 0, 0, 0);
                        }
                        if (q == 3) aS[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[0][rt], f[0][ct], aS[t], 0, 0, 0);
                    }
            }
            if constexpr (Acc) {
                int t = 0;
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int ct = rt; ct < MaxCT; ++ct, ++t) {
                        if (!(rt < RT && ct < CT)) continue;
#pragma unroll
                        for (int r = 0; r < 4; ++r) a64[t][r] += (double)aS[t][r];
                        aS[t] = floatx4{0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
        for (int pass = 0; pass < 2; ++pass) {
            int t = 0;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int ct = rt; ct < MaxCT; ++ct, ++t) {
                    if (!(rt < RT && ct < CT)) continue;
                    const int j = ct * 16 + c16;
                    if (j >= m) continue;
                    const uint32_t oj = s_oid[w][j];
                    const uint64_t tj = s_thr[w][j];
                    const float nj = Acc ? 0.f : s_nrm[w][j];
                    const double nj64 = Acc ? s_n64[w][j] : 0.0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = rt * 16 + g * 4 + r;
                        if (i >= nnew || (j < nnew && j <= i)) continue;
                        float D;
                        if constexpr (Acc) {
                            const double dot = Planes == 1 ? a64[t][r]
                                                           : a64[t][r] + ((double)aR[t][r] + (double)aQ[t][r]);
                            D = (float)((s_n64[w][i] + nj64) - 2.0 * dot);
                        } else {
                            const float dot = Planes == 1 ? aS[t][r] + 0.0f : aS[t][r] + (aR[t][r] + aQ[t][r]);
                            D = (s_nrm[w][i] + nj) - 2.0f * dot;
                        }
                        D = D > 0.f ? D : 0.f;
                        const uint64_t kb = (uint64_t)__float_as_uint(D) << 32;
                        const uint64_t ki = kb | oj, kj = kb | s_oid[w][i];
                        if (pass == 0) {
                            if (ki < s_thr[w][i]) emit_count(el, i);
                            if (kj < tj) emit_count(el, j);
                        } else {
                            if (ki < s_thr[w][i]) emit_write(v, el, i, ki);
                            if (kj < tj) emit_write(v, el, j, kj);
                        }
                    }
                }
            if (pass == 0) emit_reserve(v, el, s_pos[w], m);
        }
        wave_sync();
        emit_clear(el, m);
    }
}

template <int MaxCT, bool Acc>
static void launch_join_split_ct(const Views& v, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 g(grid_for(v.N, kJoinWaves, pass_cap(v)));
    if constexpr (!Acc) {
        if (v.u8) {
            launch_timed(k_join_split<MaxCT, 1, false, true>, g, dim3(256), 0, s, e0, e1, v);
            return;
        }
    }
    if (v.planes == 1)
        launch_timed(k_join_split<MaxCT, 1, Acc>, g, dim3(256), 0, s, e0, e1, v);
    else if (v.planes == 2)
        launch_timed(k_join_split<MaxCT, 2, Acc>, g, dim3(256), 0, s, e0, e1, v);
    else
        launch_timed(k_join_split<MaxCT, 3, Acc>, g, dim3(256), 0, s, e0, e1, v);
}

void launch_join_split(const Views& v, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (2 * v.C <= 32)
        v.acc ? launch_join_split_ct<2, true>(v, s, e0, e1) : launch_join_split_ct<2, false>(v, s, e0, e1);
    else if (2 * v.C <= 48)
        v.acc ? launch_join_split_ct<3, true>(v, s, e0, e1) : launch_join_split_ct<3, false>(v, s, e0, e1);
    else
        v.acc ? launch_join_split_ct<4, true>(v, s, e0, e1) : launch_join_split_ct<4, false>(v, s, e0, e1);
}

// ------------------------------------------------------------------ merge (a5)

constexpr int kMergeWaves = 4;
constexpr uint32_t kHubProposals = 1024;  // buckets above this are merged by a whole workgroup
constexpr int kHubWaves = 16;
constexpr int kMergeBlocks = 4096;      // partial-sum slots of k_merge
constexpr int kHubBlocks = 512;

// Ascending bitonic sort of 64 keys, one per lane.
__device__ __forceinline__ void wave_sort_keys(uint64_t& k) {
    const int lane = lane_id();
    // a distinct 32-bit proxy: the top 26 bits of the distance (non-negative
    // FP32 bits order as the values) above the lane; sorted, the full keys
    // are fetched back and runs of equal proxy distances finished on the
    // full key
    uint32_t x = (((uint32_t)(k >> 32) >> 5) << 6) | (uint32_t)lane;
    seg_sort32<64>(x);
    k = shfl64(k, (int)(x & 63u));
    for (int pass = 0; pass < 64; ++pass) {
        bool any = false;
#pragma unroll
        for (int ph = 0; ph < 2; ++ph) {
            const bool lower = (lane & 1) == ph;   // phase 0: pairs (2i, 2i+1); phase 1: (2i+1, 2i+2)
            const bool has = lower ? lane < 63 : lane >= 1;
            const uint64_t o = shfl64(k, has ? (lower ? lane + 1 : lane - 1) : lane);
            const bool sw = has && (lower ? o < k : k < o);
            k = sw ? o : k;
            any |= sw;
        }
        if (ballot(any) == 0ull) break;
    }
}

// Folds proposal keys sorted ascending into the list (key, pf): the reversed
// keys and the list give, lane by lane, the smaller key; that bitonic
// sequence holds the 64 smallest keys of both and one half-cleaner pass
// sorts it. Entries taken from the proposals find their position from the id.
__device__ __forceinline__ void fold_sorted(uint64_t pk, uint64_t& key, uint32_t& pf) {
    const int lane = lane_id();
    const uint64_t rk = shfl64(pk, 63 - lane);
    if (rk < key) {
        key = rk;
        pf = kPosUnknown;
    }
    wave_bitonic_clean(key, pf);
}

constexpr int kInsertMax = 4;   // proposals merged one by one rather than sorted

// Merges proposals q (lanes in qm; each below kth when it was taken and not
// a snapshot id; +inf in the other lanes) into the list held one entry per
// lane in (key, pf), ascending, +inf beyond K. A few are inserted one by one
// (ballot rank, shift up), skipping any no longer below the K-th key or whose
// id is already in the list (same pair, same key: the join gives a pair one
// key). More are sorted (bitonic) and folded into the list (fold_sorted).
// Repeated keys would each take a slot of the 64 smallest, so when one lands
// among the first K the fold is redone from the list as it was, with every
// key that repeats its neighbour or a list key (binary search in LDS)
// removed and the rest compacted in order (sk: 64 slots of this wave).
__device__ __forceinline__ void merge_pending(uint64_t q, uint64_t qm, int K, uint64_t& key, uint32_t& pf,
                                              uint64_t& kth, uint64_t* sk) {
    const int lane = lane_id();
    if (__popcll(qm) <= kInsertMax) {
        while (qm) {
            const int j = __ffsll((long long)qm) - 1;
            qm &= qm - 1;
            const uint64_t x = rl64(q, j);
            if (x >= kth) continue;
            if (ballot(lane < K && (uint32_t)key == (uint32_t)x)) continue;
            const int at = __popcll(ballot(lane < K && key < x));
            const uint64_t ku = shfl_up64(key, 1);
            const uint32_t pu = (uint32_t)__shfl_up((int)pf, 1);
            if (lane > at && lane < K) {
                key = ku;
                pf = pu;
            }
            if (lane == at) {
                key = x;
                pf = kPosUnknown;
            }
            kth = rl64(key, K - 1);
        }
        return;
    }
    wave_sort_keys(q);
    const uint64_t k0 = key;
    const uint32_t f0 = pf;
    fold_sorted(q, key, pf);
    const uint64_t prevk = shfl_up64(key, 1);  // all lanes take part in the shuffle
    if (ballot(lane > 0 && lane < K && key != ~0ull && prevk == key)) {
        sk[lane] = k0;
        wave_sync();
        int lo = 0;   // keys of the list below q (at most 63)
        for (int st = 32; st > 0; st >>= 1) lo += sk[lo + st - 1] < q ? st : 0;
        const uint64_t prevq = shfl_up64(q, 1);
        const bool keep = q != ~0ull && sk[lo] != q && !(lane > 0 && prevq == q);
        const uint64_t km = ballot(keep);
        wave_sync();
        sk[lane] = ~0ull;
        wave_sync();
        if (keep) sk[mbcnt(km)] = q;
        wave_sync();
        q = sk[lane];
        wave_sync();
        key = k0;
        pf = f0;
        fold_sorted(q, key, pf);
    }
    if (lane >= K) {
        key = ~0ull;
        pf = 0u;
    }
    kth = rl64(key, K - 1);
}

// Folds proposals src[c0 .. n) (chunks of 64, every `stride` elements) into
// the list. A proposal is dropped when it is not below the current K-th key
// or its id is in the snapshot list (snap: ids, lanes < K; compared by id,
// since the list's keys may come from the initial graph, whose distances are
// summed in another order than the join's). Survivors of successive chunks
// are queued in sk (64 slots of this wave) and merged when the next chunk's
// survivors do not fit and at the end, so a target whose later chunks thin
// out sorts a few full queues rather than one sparse chunk at a time; a last
// chunk with nothing queued is merged straight from the registers.
__device__ __forceinline__ void merge_chunks(const uint64_t* pks, uint32_t c0, uint32_t n, uint32_t stride,
                             int K, uint32_t snap, uint64_t& key, uint32_t& pf, uint64_t& kth,
                             uint64_t* sk) {
    const int lane = lane_id();
    int np = 0;   // queued proposals in sk[0 .. np)
    uint64_t nk = ~0ull;
    if (c0 + (uint32_t)lane < n) nk = pks[c0 + lane];
    for (;; c0 += stride) {
        const bool last = c0 >= n;
        const uint64_t pk = nk;   // NEW entries: the position is found when the id enters the list
        bool ok = false;
        uint64_t mask = 0;
        int cnt = 0;
        if (!last) {
            // next chunk in flight while this one is filtered
            nk = ~0ull;
            if (c0 + stride + (uint32_t)lane < n) nk = pks[c0 + stride + lane];
            ok = pk < kth;
            if (ballot(ok)) {
                // ids are below 2^31, so (a ^ b) - 1 has bit 31 set exactly when
                // a == b: lane-local arithmetic, no lane-mask work per entry
                const uint32_t pid = (uint32_t)pk;
                uint32_t hit = 0u;
                int k = 0;
                for (; k + 4 <= K; k += 4)
                    hit |= ((rl32(snap, k) ^ pid) - 1u) | ((rl32(snap, k + 1) ^ pid) - 1u) |
                           ((rl32(snap, k + 2) ^ pid) - 1u) | ((rl32(snap, k + 3) ^ pid) - 1u);
                for (; k < K; ++k) hit |= (rl32(snap, k) ^ pid) - 1u;
                ok &= (hit >> 31) == 0u;
                mask = ballot(ok);
                cnt = __popcll(mask);
            }
        }
        // one merge site: the last chunk with an empty queue, a queue that
        // cannot take this chunk, or the end of the input
        const bool direct = !last && np == 0 && c0 + stride >= n;
        if (direct || (np && (last || np + cnt > 64))) {
            uint64_t q = ok ? pk : ~0ull, qm = mask;
            if (!direct) {
                wave_sync();
                q = lane < np ? sk[lane] : ~0ull;
                qm = np == 64 ? ~0ull : ((1ull << np) - 1);
                wave_sync();
            }
            merge_pending(q, qm, K, key, pf, kth, sk);
            if (direct) break;
            np = 0;
            ok = ok && pk < kth;
            mask = ballot(ok);
            cnt = __popcll(mask);
        }
        if (last) break;
        if (ok) sk[np + (int)mbcnt(mask)] = pk;
        np += cnt;
    }
}

// Writes a merged row back; checks that every id names a point of the
// dataset and that no id appears twice (that would mean two different keys
// for one pair; the entries kept from the snapshot are distinct, so only
// those that entered are compared), and counts the entered ids (c_t). An
// entry entered exactly when it came from a proposal (position word
// kPosUnknown); it gets its position from the id: the dataset's first
// position plus the id (batched form), the id itself until the permutation
// has run (positions are the identity), else posof.
__device__ __forceinline__ uint64_t finish_merged_row(const Views& v, int p, uint64_t key, uint32_t pf) {
    const int lane = lane_id(), K = v.K;
    const size_t row = (size_t)p * K;
    const uint64_t em = ballot(lane < K && pf == kPosUnknown);
    const uint32_t base = v.ds ? v.dsbase[v.ds[p]] : 0u;
    const uint32_t npts = v.ds ? v.dsbase[v.ds[p] + 1] - base : (uint32_t)v.N;
    const bool lost = lane < K && (uint32_t)key >= npts;
    if (ballot(lost) && lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 512ull);
    if (lost) pf = kNewBit;   // position 0: the build reports the error after this iteration
    if (lane < K && pf == kPosUnknown) {
        const uint32_t id = (uint32_t)key;
        pf = (v.ds ? base + id : v.permuted ? (uint32_t)v.posof[id] : id) | kNewBit;
    }
    bool twice = false;
    for (uint64_t m = em; m; m &= m - 1) {
        const int e = __ffsll((long long)m) - 1;
        const uint32_t ie = rl32((uint32_t)key, e);
        twice |= lane < K && lane != e && (uint32_t)key == ie;
    }
    if (ballot(twice) && lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 8ull);
    if (lane < K) {
        v.lkey[row + lane] = key;
        v.lpos[row + lane] = pf;
        if (lane == K - 1) {   // the joins read the record when there is one
            if (v.rk)
                v.rk[row / K].kth = key;
            else
                v.kth[row / K] = key;
        }
    }
    const uint64_t c = (uint64_t)__popcll(em);
    if (v.chg && lane == 0) v.chg[row / K] = (uint32_t)c;   // batched form: changes per target
    return c;
}

// One wave per target; buckets above kHubProposals go to k_merge_hubs.
__global__ __launch_bounds__(256, 8) void k_merge(Views v) {
    if (stopped(v)) return;
    __shared__ uint64_t s_k[kMergeWaves][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int K = v.K;
    uint64_t changes = 0, props = 0, pairs = 0;
    for (int p = blockIdx.x * kMergeWaves + w; p < v.N; p += gridDim.x * kMergeWaves) {
        pairs += v.cap[p];   // e(u) of owner p: e_t without a scan
        const uint32_t base = bucket_lo(v, p);
        const uint32_t n = min(v.pcnt[p], bucket_lo(v, p + 1) - base);
        if (n == 0) continue;
        if (n > kHubProposals) {   // its bucket cursor is cleared by k_merge_hubs
            if (lane == 0) {
                const uint32_t slot = (uint32_t)atomicAdd((unsigned long long*)&v.counters[kCntHubs], 1ull);
                v.hubs[slot] = (uint32_t)p;
            }
            continue;
        }
        if (lane == 0) v.pcnt[p] = 0u;   // bucket cursors start the next iteration at zero
        const size_t row = (size_t)p * K;
        uint64_t key = lane < K ? v.lkey[row + lane] : ~0ull;
        uint32_t pf = lane < K ? v.lpos[row + lane] : 0u;
        const uint32_t snap = lane < K ? (uint32_t)key : 0xffffffffu;
        uint64_t kth = rl64(key, K - 1);
        merge_chunks(v.pkey + base, 0, n, 64, K, snap, key, pf, kth, s_k[w]);
        changes += finish_merged_row(v, p, key, pf);
        props += n;
    }
    // per-block partial sums (no same-address atomics); summed by k_finish_counters
    __shared__ uint64_t s_red[kMergeWaves][3];
    if (lane == 0) {
        s_red[w][0] = changes;
        s_red[w][1] = props;
        s_red[w][2] = pairs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, b = 0, c = 0;
        for (int i = 0; i < kMergeWaves; ++i) {
            a += s_red[i][0];
            b += s_red[i][1];
            c += s_red[i][2];
        }
        v.partial[3 * blockIdx.x] = a;
        v.partial[3 * blockIdx.x + 1] = b;
        v.partial[3 * blockIdx.x + 2] = c;
    }
}

// ---- merge with one 16-lane row per target (K <= 16)

constexpr int kSegLanes = 16;

// Ascending bitonic sort of 64-bit keys within segments of S lanes (equal
// keys allowed).
template <int S>
__device__ __forceinline__ void seg_sort64(uint64_t& k) {
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= S; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) {
            const uint64_t o = shfl_xor64(k, j);
            const bool keep_min = (size == S || (lane & size) == 0) == ((lane & j) == 0);
            k = keep_min ? (o < k ? o : k) : (k < o ? o : k);
        }
    }
}

// fold_sorted within each segment: the proposals q (ascending in the
// segment), reversed, against the list lane by lane keep the S smallest keys
// of both as a bitonic sequence, which the half-cleaners sort.
template <int S>
__device__ __forceinline__ void seg_fold(uint64_t q, uint64_t& key, uint32_t& pf) {
    const uint64_t rk = shfl_xor64(q, S - 1);
    if (rk < key) {
        key = rk;
        pf = kPosUnknown;
    }
#pragma unroll
    for (int j = S >> 1; j > 0; j >>= 1) cmpx(key, pf, j, true);
}

// finish_merged_row for the segment of target p (act: the segment holds a
// merged list): the same checks, positions, stores and count of entered
// entries; returns that count in the segment's first lane, 0 elsewhere. The
// check for an id held twice compares every lane of the segment with every
// entered lane by rotation.
__device__ __forceinline__ uint32_t finish_seg_row(const Views& v, int p, bool act, uint64_t key, uint32_t pf) {
    constexpr int S = kSegLanes;
    const int lane = lane_id(), sl = lane & (S - 1), g0 = lane & ~(S - 1), K = v.K;
    const bool in = act && sl < K;
    uint32_t base = 0u, npts = (uint32_t)v.N;
    if (act && v.ds) {
        const uint32_t ds = v.ds[p];
        base = v.dsbase[ds];
        npts = v.dsbase[ds + 1] - base;
    }
    const uint32_t id = (uint32_t)key;
    const bool entered = in && pf == kPosUnknown;
    const bool lost = in && id >= npts;
    if (ballot(lost) && lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 512ull);
    if (lost) pf = kNewBit;   // position 0: the build reports the error after this iteration
    if (in && pf == kPosUnknown) pf = (v.ds ? base + id : v.permuted ? (uint32_t)v.posof[id] : id) | kNewBit;
    const uint32_t tag = entered ? (id | 0x80000000u) : 0u;   // ids are below 2^31
    bool twice = false;
#pragma unroll
    for (int r = 1; r < S; ++r) {
        const uint32_t o = row_rot(tag, r);
        twice |= in && (o >> 31) != 0u && (o & 0x7fffffffu) == id;
    }
    if (ballot(twice) && lane == 0) atomicOr((unsigned long long*)&v.counters[kCntError], 8ull);
    if (in) {
        const size_t row = (size_t)p * K;
        v.lkey[row + sl] = key;
        v.lpos[row + sl] = pf;
        if (sl == K - 1) {
            if (v.rk)
                v.rk[p].kth = key;
            else
                v.kth[p] = key;
        }
    }
    const uint32_t c = (uint32_t)__popcll((ballot(entered) >> g0) & ((1ull << S) - 1));
    if (v.chg && act && sl == 0) v.chg[p] = c;   // batched form: changes per target
    return act && sl == 0 ? c : 0u;
}

// k_merge with four targets per wave, one per 16-lane row (K <= 16): short
// lists fill the wave and each target sorts its proposals 16 at a time within
// its row (DPP moves, no LDS crossbar), so the vector work and the memory
// latency of a wave are shared by four targets. The result is k_merge's: the K smallest distinct keys of
// the list and of the proposals below the K-th key whose id is not in the
// list as it was when the iteration began. Proposals are read, filtered and
// folded S at a time; a chunk whose fold puts one key twice among the first
// K is folded again from the list before it, with the chunk's keys that
// repeat a neighbour or a list key (binary search in LDS) removed.
__global__ __launch_bounds__(256, 8) void k_merge_seg(Views v) {
    if (stopped(v)) return;
    constexpr int S = kSegLanes, G = 64 / S;
    constexpr uint64_t kSeg = (1ull << S) - 1;
    __shared__ uint64_t s_k[kMergeWaves][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int sl = lane & (S - 1), g0 = lane & ~(S - 1), gi = lane / S;
    const int K = v.K;
    uint64_t changes = 0, props = 0, pairs = 0;   // per lane, summed over the wave at the end
    for (int pb = (blockIdx.x * kMergeWaves + w) * G; pb < v.N; pb += gridDim.x * kMergeWaves * G) {
        const int p = pb + gi;
        uint32_t base = 0u, n = 0u;
        if (p < v.N) {
            base = bucket_lo(v, p);
            n = min(v.pcnt[p], bucket_lo(v, p + 1) - base);
            if (sl == 0) pairs += v.cap[p];   // e(u) of owner p: e_t without a scan
        }
        const bool hub = n > kHubProposals;   // its bucket cursor is cleared by k_merge_hubs
        if (hub && sl == 0) {
            const uint32_t slot = (uint32_t)atomicAdd((unsigned long long*)&v.counters[kCntHubs], 1ull);
            v.hubs[slot] = (uint32_t)p;
        }
        const bool act = n > 0u && !hub;
        if (ballot(act) == 0ull) continue;
        if (act && sl == 0) v.pcnt[p] = 0u;   // bucket cursors start the next iteration at zero
        const bool in = act && sl < K;
        const size_t row = (size_t)p * K;
        uint64_t key = in ? v.lkey[row + sl] : ~0ull;
        uint32_t pf = in ? v.lpos[row + sl] : 0u;
        // snapshot ids; 0x7fffffff in the lanes beyond K matches no id
        const uint32_t snap = in ? (uint32_t)key : 0x7fffffffu;
        uint64_t kth = shfl64(key, g0 + K - 1);
        for (uint32_t c0 = 0;; c0 += S) {
            if (ballot(act && c0 < n) == 0ull) break;
            const uint64_t pk = act && c0 + (uint32_t)sl < n ? v.pkey[base + c0 + sl] : ~0ull;
            // (a ^ b) - 1 has bit 31 set exactly when a == b (both below 2^31)
            const uint32_t pid = (uint32_t)pk;
            uint32_t hit = (snap ^ pid) - 1u;   // every lane of the row against every other, by rotation
#pragma unroll
            for (int r = 1; r < S; ++r) hit |= (row_rot(snap, r) ^ pid) - 1u;
            const bool ok = pk < kth && (hit >> 31) == 0u;
            if (ballot(ok) == 0ull) continue;
            uint64_t q = ok ? pk : ~0ull;
            seg_sort64<S>(q);
            const uint64_t k0 = key;
            const uint32_t f0 = pf;
            seg_fold<S>(q, key, pf);
            const uint64_t prevk = shfl64(key, sl > 0 ? lane - 1 : lane);
            const uint64_t dm = ballot(sl > 0 && sl < K && key != ~0ull && prevk == key);
            if (dm) {
                const bool redo = ((dm >> g0) & kSeg) != 0ull;
                uint64_t* sk = s_k[w];
                sk[lane] = k0;
                wave_sync();
                int lo = 0;   // keys of the segment's list below q
#pragma unroll
                for (int st = S / 2; st > 0; st >>= 1) lo += sk[g0 + lo + st - 1] < q ? st : 0;
                const uint64_t prevq = shfl64(q, sl > 0 ? lane - 1 : lane);
                const bool keep = q != ~0ull && sk[g0 + lo] != q && !(sl > 0 && prevq == q);
                const uint64_t km = ballot(keep);
                wave_sync();
                sk[lane] = ~0ull;
                wave_sync();
                if (keep) sk[g0 + __popcll(km & ((1ull << lane) - 1) & ~((1ull << g0) - 1))] = q;
                wave_sync();
                const uint64_t qd = sk[lane];
                wave_sync();
                uint64_t k2 = k0;
                uint32_t f2 = f0;
                seg_fold<S>(qd, k2, f2);
                if (redo) {
                    key = k2;
                    pf = f2;
                }
            }
            if (sl >= K) {
                key = ~0ull;
                pf = 0u;
            }
            kth = shfl64(key, g0 + K - 1);
        }
        changes += finish_seg_row(v, p, act, key, pf);
        if (act && sl == 0) props += n;
    }
    for (int o = 32; o > 0; o >>= 1) {
        changes += shfl_xor64(changes, o);
        props += shfl_xor64(props, o);
        pairs += shfl_xor64(pairs, o);
    }
    // per-block partial sums (no same-address atomics); summed by k_finish_counters
    __shared__ uint64_t s_red[kMergeWaves][3];
    if (lane == 0) {
        s_red[w][0] = changes;
        s_red[w][1] = props;
        s_red[w][2] = pairs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, b = 0, c = 0;
        for (int i = 0; i < kMergeWaves; ++i) {
            a += s_red[i][0];
            b += s_red[i][1];
            c += s_red[i][2];
        }
        v.partial[3 * blockIdx.x] = a;
        v.partial[3 * blockIdx.x + 1] = b;
        v.partial[3 * blockIdx.x + 2] = c;
    }
}

// Counters of an iteration, by one workgroup of 1024 threads after the
// merge kernels have written their partial sums: c_t, proposals and e_t added
// up; after the iteration's last merge (last != 0; every block of a
// block-asynchronous iteration but the last adds its sums and clears the hub
// list only) all counters are copied to the host-visible slot (may be null)
// and cleared for the next iteration, and thr >= 0 sets *v.stop when
// changes < thr or a device invariant failed.
__device__ void finish_counters_block(const Views& v, uint64_t* slot, double thr, int last) {
    __shared__ uint64_t s_a[16], s_b[16], s_c[16];
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
    const uint64_t* part = v.partial;
    uint64_t a = 0, b = 0, c = 0;
    for (int i = t; i < kMergeBlocks + kHubBlocks; i += 1024) {
        a += part[3 * i];
        b += part[3 * i + 1];
        c += part[3 * i + 2];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += shfl_xor64(a, o);
        b += shfl_xor64(b, o);
        c += shfl_xor64(c, o);
    }
    if (lane == 0) {
        s_a[w] = a;
        s_b[w] = b;
        s_c[w] = c;
    }
    __syncthreads();
    if (t == 0) {
        uint64_t sa = 0, sb = 0, sc = 0;
        for (int i = 0; i < 16; ++i) {
            sa += s_a[i];
            sb += s_b[i];
            sc += s_c[i];
        }
        uint64_t* cnt = v.counters;
        cnt[kCntChanges] += sa;
        cnt[kCntProposals] += sb;
        cnt[kCntPairs2] += 2ull * sc;
        if (!last) {
            cnt[kCntHubs] = 0ull;   // the next block's merge lists its own hubs
            return;
        }
        if (slot) {
            for (int i = 0; i < kNumCounters; ++i) slot[i] = cnt[i];
            __threadfence_system();
        }
        if (thr >= 0.0 && v.stop) {
            const bool met = (double)cnt[kCntChanges] < thr || cnt[kCntError] != 0ull;
            *v.stop = met ? 1u : 0u;
        }
        for (int i = 0; i < kNumCounters; ++i) cnt[i] = 0ull;
    }
}

// Targets with large buckets: 16 waves each fold a strided share of the
// bucket into their own copy of the list; wave 0 then folds the other 15
// partial lists (from LDS) into its own. Equal to folding the whole bucket,
// since the K smallest of a union are the K smallest of the partial results.
__global__ __launch_bounds__(1024) void k_merge_hubs(Views v) {
    if (stopped(v)) return;
    __shared__ uint64_t s_k[kHubWaves][64];
    __shared__ uint64_t s_lk[kHubWaves][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int K = v.K;
    const int nh = (int)v.counters[kCntHubs];
    uint64_t changes = 0, props = 0;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int p = (int)v.hubs[h];
        const uint32_t base = bucket_lo(v, p);
        const uint32_t n = min(v.pcnt[p], bucket_lo(v, p + 1) - base);
        const size_t row = (size_t)p * K;
        uint64_t key = lane < K ? v.lkey[row + lane] : ~0ull;
        uint32_t pf = lane < K ? v.lpos[row + lane] : 0u;
        const uint32_t snap = lane < K ? (uint32_t)key : 0xffffffffu;
        uint64_t kth = rl64(key, K - 1);
        merge_chunks(v.pkey + base, (uint32_t)w * 64, n, kHubWaves * 64, K, snap, key, pf, kth, s_k[w]);
        s_lk[w][lane] = key;
        __syncthreads();
        if (w == 0) {
            // the other partial lists: their snapshot ids are dropped by the fold, so
            // every entry that gets through came from a proposal (NEW, position by id)
            merge_chunks(&s_lk[1][0], 0, (kHubWaves - 1) * 64, 64, K, snap, key, pf, kth, s_k[0]);
            changes += finish_merged_row(v, p, key, pf);
            props += n;
        }
        __syncthreads();
        if (threadIdx.x == 0) v.pcnt[p] = 0u;   // every wave has read it
    }
    if (w == 0 && lane == 0) {
        v.partial[3 * (kMergeBlocks + blockIdx.x)] = changes;
        v.partial[3 * (kMergeBlocks + blockIdx.x) + 1] = props;
        v.partial[3 * (kMergeBlocks + blockIdx.x) + 2] = 0;
    }
}

void launch_merge(const Views& v, hipStream_t s) {
    // rows of 16 lanes for short lists; at larger K one wave per target
    // sorts more proposals at once, which measured faster there
    if (v.K <= kSegLanes)
        hipLaunchKernelGGL(k_merge_seg, dim3(kMergeBlocks), dim3(256), 0, s, v);
    else
        hipLaunchKernelGGL(k_merge, dim3(kMergeBlocks), dim3(256), 0, s, v);
    hipLaunchKernelGGL(k_merge_hubs, dim3(kHubBlocks), dim3(1024), 0, s, v);
}

__global__ __launch_bounds__(1024) void k_finish_counters(Views v, uint64_t* slot, double thr, int last) {
    if (stopped(v)) return;
    finish_counters_block(v, slot, thr, last);
}

void launch_finish_counters(const Views& v, hipStream_t s, hipEvent_t e1, uint64_t* slot, double thr, int last) {
    launch_timed(k_finish_counters, dim3(1), dim3(1024), 0, s, nullptr, e1, v, slot, thr, last);
}

size_t partial_words() { return 3 * (size_t)(kMergeBlocks + kHubBlocks); }



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
        const int a = min((int)(nn & 0xffffu), C), b = min((int)(nn >> 16), C);   // cand holds 2C
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

// ------------------------------------------------------------------ batched form (a10)
//
// Many independent datasets share one position space (each a contiguous
// range); every kernel above is per node and never follows an edge out of a
// node's own dataset, so one launch advances every active dataset by one
// iteration. Each dataset keeps its seed (init/sample stream states), its
// iteration counter, its stop rule and its statistics on the device; nothing
// is read back, so the whole build can be captured in one graph.

// one workgroup per dataset: dataset index, local ids, padded rows
// Datasets along x, kBatchSetupSplit workgroups per dataset along y (a
// dataset of thousands of rows is copied by that many workgroups, not one).
constexpr int kBatchSetupSplit = 16;

__global__ void k_batch_setup(Views v) {
    const uint32_t ny = gridDim.y, y = blockIdx.y;
    for (int i = blockIdx.x; i < v.nds; i += gridDim.x) {
        const uint32_t b = v.dsbase[i], e = v.dsbase[i + 1];
        const int d = v.in_d[i];
        const float* X = v.in_X[i];
        uint32_t* dsw = const_cast<uint32_t*>(v.ds);
        for (uint32_t p = b + y * blockDim.x + threadIdx.x; p < e; p += ny * blockDim.x) {
            dsw[p] = (uint32_t)i;
            v.orig[p] = (int32_t)(p - b);
            v.posof[p] = (int32_t)(p - b);
        }
        // rows by waves, columns by lanes (no division per element)
        bool bad = false;
        const int lane = lane_id(), wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
        for (uint32_t r = y * nw + wv; r < e - b; r += ny * nw) {
            for (int c = lane; c < v.dp; c += 64) {
                const float x = c < d ? X[(size_t)r * d + c] : 0.f;
                bad |= (__float_as_uint(x) & 0x7f800000u) == 0x7f800000u;
                v.Xp[((size_t)b + r) * v.dp + c] = x;
            }
        }
        if (bad) flag_or(&v.counters[kCntNonFinite], 1ull);
        if (y == 0 && threadIdx.x == 0) {
            v.active[i] = 1u;
            v.ds_iters[i] = 0;
            v.ds_conv[i] = 0;
        }
    }
}

void launch_batch_setup(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_setup, dim3(v.nds < 4096 ? v.nds : 4096, kBatchSetupSplit), dim3(256), 0, s, v);
}

// after iteration t: per-dataset e_t and c_t from the scans over its range,
// then the stop rule c_t < delta*N_i*K, or t = T_max. One workgroup: once no
// dataset of the group is active it sets the group's stop word, and every
// later iteration kernel of the group returns at entry.
__global__ __launch_bounds__(1024) void k_batch_step(Views v, int t, int T_max, int K, double delta) {
    int alive = 0;
    for (int i = threadIdx.x; i < v.nds; i += blockDim.x) {
        if (!v.active[i]) continue;
        const uint32_t b = v.dsbase[i], e = v.dsbase[i + 1];
        const int64_t ev = (int64_t)(v.poff[e] - v.poff[b]);
        const int64_t ch = (int64_t)(v.chgoff[e] - v.chgoff[b]);
        v.ds_stats[((size_t)i * T_max + (t - 1)) * 2] = ev;
        v.ds_stats[((size_t)i * T_max + (t - 1)) * 2 + 1] = ch;
        v.ds_iters[i] = t;
        if ((double)ch < delta * (double)(e - b) * (double)K) {
            v.ds_conv[i] = 1;
            v.active[i] = 0u;
        } else if (t >= T_max) {
            v.active[i] = 0u;
        } else {
            alive = 1;
        }
    }
    alive = __syncthreads_or(alive);
    if (threadIdx.x == 0 && v.stop) *v.stop = alive ? 0u : 1u;
}

void launch_batch_step(const Views& v, int t, int T_max, int K, double delta, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_step, dim3(1), dim3(1024), 0, s, v, t, T_max, K, delta);
}

// per-dataset outputs: rows sorted by (distance, local id)
__global__ void k_batch_finalize(Views v) {
    const int64_t NK = (int64_t)v.N * v.K;
    const double rk = 1.0 / v.K;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < NK; e += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)udiv((uint32_t)e, (uint32_t)v.K, rk), k = (int)(e - (int64_t)p * v.K);
        const uint32_t i = v.ds[p];
        const size_t o = (size_t)(p - (int)v.dsbase[i]) * v.K + k;
        const uint64_t key = v.lkey[e];
        v.out_ids[i][o] = (int32_t)(uint32_t)key;
        v.out_dists[i][o] = __uint_as_float((uint32_t)(key >> 32));
    }
}

void launch_batch_finalize(const Views& v, hipStream_t s) {
    const int64_t NK = (int64_t)v.N * v.K;
    hipLaunchKernelGGL(k_batch_finalize, dim3(grid_for(NK, 256, 1 << 16)), dim3(256), 0, s, v);
}

// ------------------------------------------------------------------ permutation (a7)
//
// Sec. 3.2 reorders the points once, early, so that points close in the data
// space are close in memory; its greedy Alg. 1 is one sequential pass. The
// device version clusters the current K-NN graph with Boruvka-style hooking:
// at every level each component picks its cheapest edge (distance, entry
// index) to another component among the first kPermEdges entries of its
// members' lists, both endpoints competing for it, and hooks into the other
// component (the smaller label stays root when two components pick the same
// edge, the only possible cycle). The hook forest is laid out in post-order
// with the children of a node ordered by decreasing hook level, so every
// component of every level occupies a contiguous range of positions. The
// permutation is invisible in the results: hashes and tie-breaks use
// original ids.
constexpr uint32_t kNoLevel = 0xffffffffu;
constexpr int kPermEdges = 8;

__global__ void k_perm_init(Views v) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < v.N; p += gridDim.x * blockDim.x) {
        v.comp[p] = p;
        v.par[p] = p;
        v.lvl[p] = kNoLevel;
        v.size[p] = 1u;
        v.cur[p] = 0u;
        v.best[p] = ~0ull;
        v.pdone[p] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x < 4) v.flag[threadIdx.x] = 0u;
}

// flag[0]: clustering finished (a level hooked nothing); flag[1]: a hook happened this level.
// Each component takes its cheapest incident edge (either end) among the
// first kPermEdges list entries of its points; edge key (D, entry index).
// One thread per point: the point's own component gets the minimum of its
// edges in one update, the other ends one each; an atomic is issued only
// when it can lower the current value (unconditional atomics on the few
// words of large components serialise: 3x slower, measured). Components only
// merge, so a point whose scanned edges all lie inside its component stays
// so at every later level: it is marked and skipped from then on (it would
// add nothing). At level 0 every point is its own component, so the labels
// are not read.
__global__ void k_perm_edges(Views v, uint32_t level) {
    if (v.flag[0]) return;
    const int E = min(v.K, kPermEdges);
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < v.N; u += gridDim.x * blockDim.x) {
        if (v.pdone[u]) continue;
        const int cu = level ? v.comp[u] : u;
        uint64_t mine = ~0ull;
        for (int k = 0; k < E; ++k) {
            const uint32_t e = (uint32_t)u * (uint32_t)v.K + (uint32_t)k;
            const int pv = (int)(v.lpos[e] & kPosMask);
            const int cv = level ? v.comp[pv] : pv;
            if (cu == cv) continue;
            const uint64_t key = ((v.lkey[e] >> 32) << 32) | e;
            mine = key < mine ? key : mine;
            if (key < v.best[cv]) atomicMin((unsigned long long*)&v.best[cv], (unsigned long long)key);
        }
        if (mine == ~0ull)
            v.pdone[u] = 1u;
        else if (mine < v.best[cu])
            atomicMin((unsigned long long*)&v.best[cu], (unsigned long long)mine);
    }
}

__global__ void k_perm_hook(Views v, uint32_t level) {
    if (v.flag[0]) return;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < v.N; c += gridDim.x * blockDim.x) {
        int jump = c;
        if (v.comp[c] == c) {
            const uint64_t b = v.best[c];
            if (b != ~0ull) {
                const uint32_t e = (uint32_t)b;
                const int u = (int)(e / (uint32_t)v.K);
                const int pv = (int)(v.lpos[e] & kPosMask);
                const int cu = v.comp[u];
                const int other = cu == c ? v.comp[pv] : cu;
                const bool mutual = v.best[other] == b;
                if (!(mutual && c < other)) {
                    v.par[c] = other;
                    v.lvl[c] = level;
                    jump = other;
                    v.flag[1] = 1u;
                }
            }
        }
        v.comp2[c] = jump;
    }
}

// pointer jumping among this level's roots: comp2 converges to the new root.
// A root that hooked at this level takes that new root as its parent, so the
// hooks of one level form stars (a chain A->B->C within one level would make
// the subtree sizes depend on the order in which the level is summed).
__global__ void k_perm_jump(Views v, uint32_t level) {
    if (v.flag[0]) return;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < v.N; c += gridDim.x * blockDim.x) {
        if (v.comp[c] != c) continue;
        int x = v.comp2[c];
        // hook chains among one level's roots are acyclic (two components that
        // pick the same edge keep the smaller label as root); the step cap only
        // turns a violated invariant into an error instead of a spin
        int steps = 0;
        for (; steps < 4096; ++steps) {
            const int y = v.comp2[x];
            if (y == x) break;
            x = y;
        }
        if (steps == 4096) atomicOr((unsigned long long*)&v.counters[kCntError], 32ull);
        v.comp2[c] = x;
        if (v.lvl[c] == level) v.par[c] = x;
    }
}

__global__ void k_perm_relabel(Views v) {
    if (v.flag[0]) return;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < v.N; p += gridDim.x * blockDim.x) {
        v.comp[p] = v.comp2[v.comp[p]];
        v.best[p] = ~0ull;
    }
}

__global__ void k_perm_level_end(Views v) {
    if (v.flag[0]) return;
    if (!v.flag[1]) v.flag[0] = 1u;
    v.flag[1] = 0u;
    v.flag[2] += 1u;  // levels run
}

__global__ void k_perm_sizes(Views v, uint32_t level) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < v.N; c += gridDim.x * blockDim.x)
        if (v.lvl[c] == level) atomicAdd(&v.size[v.par[c]], v.size[c]);
}

__global__ void k_perm_rootsz(Views v) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < v.N; c += gridDim.x * blockDim.x)
        v.cur[c] = v.lvl[c] == kNoLevel ? v.size[c] : 0u;
}

__global__ void k_perm_clear_cur(Views v) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < v.N; c += gridDim.x * blockDim.x) v.cur[c] = 0u;
}

// children get the next free block of their parent's range, highest hook level first
__global__ void k_perm_offsets(Views v, uint32_t level) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < v.N; c += gridDim.x * blockDim.x)
        if (v.lvl[c] == level) {
            const int pa = v.par[c];
            v.offs[c] = v.offs[pa] + atomicAdd(&v.cur[pa], v.size[c]);
        }
}

// post-order: a node sits at the end of its subtree's range
__global__ void k_perm_newpos(Views v) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < v.N; c += gridDim.x * blockDim.x)
        v.newpos[c] = (int32_t)(v.offs[c] + v.size[c] - 1u);
}

// FP32 rows are moved unless the split form uses one plane (then nothing
// reads them and they were never written).
__device__ __forceinline__ bool fp32_rows_used(const Views& v) { return !(v.Xs && v.planes == 1); }

__global__ void k_perm_rows(Views v) {
    const int dp4 = fp32_rows_used(v) ? v.dp >> 2 : 1;
    const int64_t total = (int64_t)v.N * dp4;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(i / dp4), c = (int)(i - (int64_t)p * dp4);
        const int q = v.newpos[p];
        if (q < 0 || q >= v.N) {
            atomicOr((unsigned long long*)&v.counters[kCntError], 64ull);
            continue;
        }
        if (fp32_rows_used(v))
            reinterpret_cast<float4*>(v.Xp2 + (size_t)q * v.dp)[c] =
                reinterpret_cast<const float4*>(v.Xp + (size_t)p * v.dp)[c];
        if (v.rk && c == 0) v.rk2[q].x = v.rk[p].x;
        if (c == 0) {
            v.orig2[q] = v.orig[p];
            v.nrm2[q] = v.nrm[p];
            if (v.nrm64) v.nrm64_2[q] = v.nrm64[p];
        }
    }
}

__global__ void k_perm_rows_bf16(Views v) {
    const int dp8 = v.dp >> 3;   // 16-byte groups of 8 BF16 values (dp % 32 == 0)
    const int64_t total = (int64_t)v.N * dp8;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(i / dp8), c = (int)(i - (int64_t)p * dp8);
        const int q = v.newpos[p];
        if (q < 0 || q >= v.N) continue;  // reported by k_perm_rows
        reinterpret_cast<uint4*>(v.Xb2 + (size_t)q * v.dp)[c] = reinterpret_cast<const uint4*>(v.Xb + (size_t)p * v.dp)[c];
        if (c == 0) v.nb2[q] = v.nb[p];
    }
}

__global__ void k_perm_rows_split(Views v) {
    const int dp8 = v.dp >> 3;   // 16-byte groups per plane row (dp % 32 == 0)
    const int64_t per = (int64_t)v.N * dp8, total = (int64_t)v.planes * per;   // planes in use
    const size_t plane = (size_t)v.N * v.dp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(i / per);
        const int64_t r = i - (int64_t)q * per;
        const int p = (int)(r / dp8), c = (int)(r - (int64_t)p * dp8);
        const int np = v.newpos[p];
        if (np < 0 || np >= v.N) continue;  // reported by k_perm_rows
        reinterpret_cast<uint4*>(v.Xs2 + q * plane + (size_t)np * v.dp)[c] =
            reinterpret_cast<const uint4*>(v.Xs + q * plane + (size_t)p * v.dp)[c];
    }
}

__global__ void k_perm_rows_u8(Views v) {
    const int dp8 = v.dp >> 3;   // 8-byte groups per byte row
    const int64_t total = (int64_t)v.N * dp8;
    const size_t plane = (size_t)v.N * v.dp;
    const uint2* src = reinterpret_cast<const uint2*>(reinterpret_cast<const uint8_t*>(v.Xs + plane));
    uint2* dst = reinterpret_cast<uint2*>(reinterpret_cast<uint8_t*>(v.Xs2 + plane));
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(i / dp8), c = (int)(i - (int64_t)p * dp8);
        const int np = v.newpos[p];
        if (np < 0 || np >= v.N) continue;  // reported by k_perm_rows
        dst[(size_t)np * dp8 + c] = src[(size_t)p * dp8 + c];
    }
}

__global__ void k_perm_lists(Views v) {
    const int64_t NK = (int64_t)v.N * v.K;
    const double rk = 1.0 / v.K;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < NK; e += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)udiv((uint32_t)e, (uint32_t)v.K, rk), k = (int)(e - (int64_t)p * v.K);
        const int q = v.newpos[p];
        const uint32_t pf = v.lpos[e];
        const int qn = v.newpos[pf & kPosMask];
        if (q < 0 || q >= v.N || qn < 0 || qn >= v.N) {
            atomicOr((unsigned long long*)&v.counters[kCntError], 64ull);
            continue;
        }
        const size_t to = (size_t)q * v.K + k;
        v.lkey2[to] = v.lkey[e];
        v.lpos2[to] = (uint32_t)qn | (pf & kNewBit);
        if (k == v.K - 1) {
            if (v.rk)
                v.rk2[q].kth = v.lkey[e];
            else
                v.kth2[q] = v.lkey[e];
        }
    }
}

__global__ void k_perm_posof(Views v) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < v.N; p += gridDim.x * blockDim.x) v.posof[v.orig[p]] = p;
}

int perm_levels_max() { return 32; }

void launch_perm_begin(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_init, dim3(grid_for(v.N, 256, 8192)), dim3(256), 0, s, v);
}

void launch_perm_level(const Views& v, uint32_t level, hipStream_t s) {
    const int g = grid_for(v.N, 256, 8192);
    hipLaunchKernelGGL(k_perm_edges, dim3(grid_for(v.N, 256, 16384)), dim3(256), 0, s, v, level);
    hipLaunchKernelGGL(k_perm_hook, dim3(g), dim3(256), 0, s, v, level);
    hipLaunchKernelGGL(k_perm_jump, dim3(g), dim3(256), 0, s, v, level);
    hipLaunchKernelGGL(k_perm_relabel, dim3(g), dim3(256), 0, s, v);
    hipLaunchKernelGGL(k_perm_level_end, dim3(1), dim3(1), 0, s, v);
}

void launch_perm_finish(const Views& v, uint32_t levels, hipStream_t s) {
    const int g = grid_for(v.N, 256, 8192);
    for (uint32_t l = 0; l < levels; ++l) hipLaunchKernelGGL(k_perm_sizes, dim3(g), dim3(256), 0, s, v, l);
    hipLaunchKernelGGL(k_perm_rootsz, dim3(g), dim3(256), 0, s, v);
    launch_scan(v.cur, v.offs, v.N, v.scan_tmp, s);
    hipLaunchKernelGGL(k_perm_clear_cur, dim3(g), dim3(256), 0, s, v);
    for (int l = (int)levels - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_perm_offsets, dim3(g), dim3(256), 0, s, v, (uint32_t)l);
    hipLaunchKernelGGL(k_perm_newpos, dim3(g), dim3(256), 0, s, v);
    hipLaunchKernelGGL(k_perm_rows, dim3(grid_for((int64_t)v.N * (v.dp >> 2), 256, 16384)), dim3(256), 0, s, v);
    hipLaunchKernelGGL(k_perm_lists, dim3(grid_for((int64_t)v.N * v.K, 256, 16384)), dim3(256), 0, s, v);
    if (v.Xb)
        hipLaunchKernelGGL(k_perm_rows_bf16, dim3(grid_for((int64_t)v.N * (v.dp >> 3), 256, 16384)), dim3(256), 0, s,
                           v);
    if (v.Xs)
        hipLaunchKernelGGL(k_perm_rows_split, dim3(grid_for(3 * (int64_t)v.N * (v.dp >> 3), 256, 16384)), dim3(256),
                           0, s, v);
    if (v.u8)
        hipLaunchKernelGGL(k_perm_rows_u8, dim3(grid_for((int64_t)v.N * (v.dp >> 3), 256, 16384)), dim3(256), 0, s, v);
}

void launch_perm_posof(const Views& v, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_posof, dim3(grid_for(v.N, 256, 8192)), dim3(256), 0, s, v);
}

}  // namespace knng
