// Internal interface between the host orchestrator (knng_api.hip) and the
// device kernels (knng_kernels.hip). Not installed; the public ABI is knng.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knng {

constexpr uint32_t kNewBit = 0x80000000u;   // flag bit in a list entry's position word
constexpr uint32_t kPosMask = 0x7fffffffu;
constexpr uint32_t kPosUnknown = 0xffffffffu;  // merge: NEW entry whose position is found from its id
constexpr int kWave = 64;
constexpr int kSelectStage = 512;           // pool entries a select wave stages in LDS
// layout-pass bits (counter kCntSplit) that make FP32 Gram sums inexact
constexpr uint64_t kLayoutInexact = 4u | 8u;

// Device counters of one iteration (uint64 slots).
enum Counter : int {
    kCntChanges = 0,     // c_t
    kCntProposals = 1,   // proposals that passed the snapshot filter
    kCntPairs2 = 2,      // 2 * e_t
    kCntError = 3,       // nonzero: a device-side invariant failed
    kCntNonFinite = 4,   // nonzero: X holds a NaN or an infinity
    kCntSplit = 5,       // layout pass: bit 0 some x2 != 0, bit 1 some x3 != 0 (split-BF16 copies),
                         // bit 2 some value is not an integer, bit 3 some squared norm exceeds 2^23,
                         // bit 4 some value is outside 0..255
    kCntHubs = 6,        // targets whose proposal bucket is merged by a workgroup
    kCntRescored = 7,    // precision form: pairs that passed the BF16 screen and were rescored
    kNumCounters = 8
};

// How a kernel outside the join computes a distance: the formula of the
// join of the resolved path (exactly the same value for the VALU form).
enum DistMode : int {
    kDistDirect = 0,   // sum_j (x_j - y_j)^2, FP32 (VALU path)
    kDistGram = 1      // FP32 Gram form (matrix paths)
};

// Views of the caller's workspace, carved by the host.
// Low-d direct form (rows of 4 floats): a point's padded row and its list's
// K-th key in one 32-byte record, so that the join's member gather (the row
// and the snapshot key) touches one cache line instead of two.
struct RowKey {
    float4 x;
    uint64_t kth;
    uint64_t pad;
};

struct Views {
    int N, d, dp, K, C;
    int turbo;          // 1: turbosampling coin in the sampling step (Sec. 3.1)
    float* Xp;          // [N, dp] rows in position order, zero padded
    float* nrm;         // [N] squared norms (Gram path), FP32
    double* nrm64;      // [N] squared norms in FP64 (Gram path)
    int acc;            // Gram path: 1 = FP64 accumulation per 32 dimensions (FP32 sums of X not exact)
    uint16_t* Xb;       // [N, dp] BF16 copies of the rows (precision form), else null
    float2* nb;         // [N] BF16 rows: {squared norm, norm of the rounding error bf16(x) - x}
    uint16_t* Xs;       // [3, N, dp] split-BF16 copies x = x1 + x2 + x3 (split form), else null
    int planes;         // split form: leading planes the join reads (1..3; the rest are all zero)
    int u8;             // split form on 8-bit data (integers 0..255, FP32 sums exact): the join and
                        // the initial distances read byte rows, Xs + N dp (the unused second plane)
    int32_t* orig;      // [N] position -> original id
    int32_t* posof;     // [N] original id -> position
    int permuted;       // 0 until the graph-ordered permutation ran: position = original id
    int blk_on, blk_lo, blk_hi;   // block-asynchronous iteration: only owners with original
                                  // ids in [blk_lo, blk_hi) sample and join (blk_on != 0)
    int grid_cap;       // > 0: workgroups of the select and join passes (grid-stride loops over the
                        // owners); 0: one workgroup per four owners, at most 65536
    uint64_t* lkey;     // [N, K] (f32 bits of D << 32) | original id, rows ascending
    uint32_t* lpos;     // [N, K] position of the neighbour | kNewBit
    uint64_t* kth;      // [N] the list's K-th key (lkey[p, K-1]), written with the list: the joins'
                        // snapshot filter reads 8 bytes per member instead of a line of its list
    RowKey* rk;         // [N] low-d direct form only (dp == 4, single builds): rows and K-th keys
                        // together; the K-th keys are then kept here instead of in kth; else null
    uint32_t* rdeg;     // [N] reverse in-degree
    uint32_t* roff;     // [N + 1] reverse bucket offsets
    uint32_t* rcur;     // [N] reverse bucket cursors
    uint4* rev;         // [N * K] reverse entries {w, orig src, pos src | flag, 0}
    // counting-sort reverse bucketing (rev_S = 0: per-entry atomics instead)
    int rev_shift;      // super-bucket = 2^rev_shift consecutive target positions
    int rev_S;          // super-buckets
    int rev_B;          // blocks of rev_E list entries
    int rev_E;
    uint32_t* rev_h;    // [rev_S * rev_B] counts, super-bucket major
    uint32_t* rev_hs;   // [rev_S * rev_B + 1] their exclusive scan
    uint32_t* rev_tmp;  // scan scratch
    uint2* cand;        // [N, 2C] sampled members {orig, pos}: new then old
    uint32_t* nn;       // [N] n_new | n_old << 16
    uint32_t* big;      // [N] 1: the owner's pool has more than 64 entries
    uint32_t* hubs;     // [N] targets with large proposal buckets
    uint32_t* cap;      // [N] pairs e(u) each owner joins this iteration
    uint32_t* poff;     // [N + 1] exclusive scan of cap (e_t = poff[N])
    uint32_t* pcnt;     // [N] proposal bucket cursors (buckets: bucket_lo)
    uint64_t* pkey;     // [Pmax = 2 N K (2C - 1)] proposal keys, bucketed by target
    uint32_t* scan_tmp; // scan scratch
    uint64_t* counters; // [kNumCounters]
    uint64_t* partial;  // [partial_words()] per-block partial sums of the merge
    // batched form (null for a single build): datasets occupy contiguous position ranges
    int nds;                    // number of datasets
    const uint32_t* ds;         // [N] dataset of each position
    const uint32_t* dsbase;     // [nds + 1] first position of each dataset
    uint32_t* active;           // [nds] 1 while the dataset iterates
    const uint64_t* st_init;    // [nds] init stream state of each dataset's seed
    const uint64_t* st_table;   // [T_max, nds] sample stream state of iteration t (row t-1)
    uint32_t* chg;              // [N] ids that entered each target's list this iteration
    uint32_t* chgoff;           // [N + 1] scan of chg
    int32_t* const* out_ids;    // [nds] per-dataset outputs
    float* const* out_dists;    // [nds]
    const float* const* in_X;   // [nds] per-dataset inputs
    const int32_t* in_d;        // [nds]
    int32_t* ds_iters;          // [nds] iterations run
    int32_t* ds_conv;           // [nds] 1 if the stop rule held
    int64_t* ds_stats;          // [nds, T_max, 2] evals and changes per iteration
    // permutation scratch
    int32_t* comp;      // [N] component label (a position) of each point
    int32_t* comp2;     // [N] pointer-jumping scratch
    uint8_t* pdone;     // [N] 1 once every scanned list edge of the point lies inside its component
    int32_t* par;       // [N] hook parent
    uint32_t* lvl;      // [N] hook level (kNoLevel: never hooked)
    uint64_t* best;     // [N] cheapest outgoing edge per component
    uint32_t* size;     // [N] subtree size in the hook forest
    uint32_t* offs;     // [N] first position of the subtree
    uint32_t* cur;      // [N] allocation cursor
    int32_t* newpos;    // [N]
    uint64_t* lkey2;    // [N, K] permuted copies (swapped with the originals)
    uint32_t* lpos2;    // [N, K]
    uint64_t* kth2;     // [N]
    RowKey* rk2;        // [N]
    float* Xp2;         // [N, dp]
    float* nrm2;        // [N]
    double* nrm64_2;    // [N]
    uint16_t* Xb2;      // [N, dp]
    float2* nb2;        // [N]
    uint16_t* Xs2;      // [3, N, dp]
    int32_t* orig2;     // [N]
    uint32_t* flag;     // small device flags
    uint32_t* stop;     // single build: set when the stop rule held (or a device
                        // invariant failed); the kernels of an iteration enqueued
                        // ahead then return at once. Null in the batched form.
};

size_t scan_tmp_words(int n);
size_t partial_words();

// kernels (launchers; all enqueue on `s`). Launchers that bound a timed phase
// take optional events e0 / e1, stamped at the start / end of their first /
// last kernel by the dispatch itself (no marker packets between kernels).
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s, const uint32_t* stop = nullptr);
void launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s, const uint32_t* stop = nullptr);
void launch_pad_rows(const float* X, const Views& v, hipStream_t s);
void launch_norms(const Views& v, hipStream_t s);
void launch_init(const Views& v, uint64_t st_init, int mode, hipStream_t s);
void launch_load_rows(const Views& v, const int32_t* ids, const float* dists, const uint8_t* flags, int mode,
                      hipStream_t s);
void launch_make_split(const Views& v, hipStream_t s);
// one pass over X for the MFMA forms: padded rows, norms, identity positions,
// finiteness check and (split != 0) the split-BF16 planes
void launch_prep(const float* X, const Views& v, int split, hipStream_t s);
// split form with planes > 1 (or a reader of the FP32 rows): padded FP32 rows
// and planes 2 and 3
void launch_prep_rest(const float* X, const Views& v, hipStream_t s);
void launch_join_split(const Views& v, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_rev_hist(const Views& v, hipStream_t s, hipEvent_t e0 = nullptr);
// batched form
void launch_batch_setup(const Views& v, hipStream_t s);
void launch_batch_step(const Views& v, int t, int T_max, int K, double delta, hipStream_t s);
void launch_batch_finalize(const Views& v, hipStream_t s);
void launch_scan(const uint32_t* in, uint32_t* out, int n, uint32_t* tmp, hipStream_t s,
                 const uint32_t* stop = nullptr);
void launch_rev_scatter(const Views& v, uint64_t st_sample, int t, hipStream_t s);
// reverse buckets (roff, rev) by the counting sort; staging in the proposal buffer
void launch_rev_partition(const Views& v, uint64_t st_sample, int t, hipStream_t s, hipEvent_t e0 = nullptr);
constexpr int kRevMaxS = 8192;    // super-buckets (LDS counters of one block)
constexpr int kRevMaxShift = 12;  // largest super-bucket: 4096 positions
void launch_select(const Views& v, uint64_t st_sample, int t, hipStream_t s);
void launch_join_valu(const Views& v, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_join_mfma(const Views& v, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_make_bf16(const Views& v, hipStream_t s);
void launch_join_bf16(const Views& v, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_merge(const Views& v, hipStream_t s);
// Sums the merge's partials into the counters (single builds); slot
// (host-visible, may be null) receives a copy of all counters, which are then
// cleared for the next iteration; thr >= 0 sets *v.stop when changes < thr or
// a device invariant failed.
void launch_finish_counters(const Views& v, hipStream_t s, hipEvent_t e1, uint64_t* slot, double thr, int last = 1);
constexpr int kStopFlag = 12;   // index of the stop word in the device flags
void launch_finalize(const Views& v, int32_t* ids, float* dists, uint8_t* flags, hipStream_t s);
void launch_export_samples(const Views& v, int32_t* dnew, int32_t* dold, int32_t* counts, hipStream_t s);
int perm_levels_max();
void launch_perm_begin(const Views& v, hipStream_t s);
void launch_perm_level(const Views& v, uint32_t level, hipStream_t s);
void launch_perm_finish(const Views& v, uint32_t levels, hipStream_t s);
void launch_perm_posof(const Views& v, hipStream_t s);
bool join_valu_fits(const Views& v);

}  // namespace knng
