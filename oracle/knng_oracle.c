/*
 * FP64 CPU oracle for synchronous, seeded NN-Descent with the squared-l2 metric.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path links, loads or calls
 * this file: it is used by tests/, by the smoke check and by the CPU-baseline
 * leg of bench.py. It shares no code, header or table with the HIP library.
 *
 * Method: Kluser, Bokstaller, Rutz, Buner, "Fast single-core K-Nearest Neighbor
 * Graph computation" (arXiv 2112.06630).
 *   - Problem (K-NNG as a directed simple graph, self excluded): Sec. 2.
 *   - Random initial graph, select/calculate iterations, stop on few changes: Sec. 2.
 *   - Neighbourhood = forward list union reverse list, fused one-pass weighted
 *     sampling ("keep the rho*k smallest uniform weights"): Sec. 3.1.
 *   - Squared l2 distance, square root omitted: Sec. 3.3 and Sec. 4.
 *
 * The paper defers the new/old bookkeeping and the stop rule to Dong et al.;
 * the readings taken here (synchronous snapshot, new/old flags, per-pair hashed
 * weights, (distance, id) tie-break, c_t < delta*N*K) are stated at each step
 * below.
 *
 * Everything is plain and sequential per node; OpenMP only splits independent
 * nodes across threads, and every reduction is done in a fixed order, so the
 * result does not depend on the thread count.
 *
 * Error behaviour: functions return 0 on success, a negative value on invalid
 * arguments (-1) or allocation failure (-2).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OLD 0
#define ORC_NEW 1
#define ORC_WEIGHTED 0 /* sampling rules (Sec. 3.1): heap (smallest weights) */
#define ORC_TURBO 1    /* turbosampling (Bernoulli coin) */

/* ---------------------------------------------------------------- hashing
 * Counter-based random numbers. mix64 is the SplitMix64 output function
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014): xor-shift 30, multiply, xor-shift 27, multiply, xor-shift 31.
 */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* H(seed, tag, t, a, b): tag 1 = initial graph, tag 2 = sampling weights. */
uint64_t orc_hash(uint64_t seed, uint64_t tag, uint64_t t, uint32_t a, uint32_t b)
{
    uint64_t s = orc_mix64(seed + 0x9E3779B97F4A7C15ULL * (tag + 1));
    uint64_t st = orc_mix64(s ^ t);
    return orc_mix64(st ^ (((uint64_t)a << 32) | (uint64_t)b));
}

/* Per-flag sample cap C = min(K, max(1, ceil(rho*K))): Sec. 3.1 bounds each
 * neighbourhood by rho*k; the ceiling is the reading for non-integer rho*K. */
int32_t orc_cap(int32_t K, double rho)
{
    double r = ceil(rho * (double)K);
    int32_t c = (int32_t)r;
    if (c < 1) c = 1;
    if (c > K) c = K;
    return c;
}

/* Squared l2 distance (Sec. 3.3: the square root is omitted), float32 inputs
 * widened exactly to double and summed left to right. */
double orc_dist(const float *X, int64_t d, int64_t p, int64_t q)
{
    const float *a = X + p * d, *b = X + q * d;
    double s = 0.0;
    for (int64_t j = 0; j < d; ++j) {
        double t = (double)a[j] - (double)b[j];
        s += t * t;
    }
    return s;
}

/* Lexicographic (distance, id) order: the tie-break reading. */
static int key_less(double da, int32_t ia, double db, int32_t ib)
{
    return da < db || (da == db && ia < ib);
}

typedef struct { double dist; int32_t id; uint8_t flag; } orc_entry;

static int cmp_entry(const void *x, const void *y)
{
    const orc_entry *a = (const orc_entry *)x, *b = (const orc_entry *)y;
    if (key_less(a->dist, a->id, b->dist, b->id)) return -1;
    if (key_less(b->dist, b->id, a->dist, a->id)) return 1;
    return 0;
}

/* (id, distance) order: groups repeated proposals of one id, smallest first */
static int cmp_entry_by_id(const void *x, const void *y)
{
    const orc_entry *a = (const orc_entry *)x, *b = (const orc_entry *)y;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    if (a->dist != b->dist) return a->dist < b->dist ? -1 : 1;
    return 0;
}

/* ---------------------------------------------------------------- step 1: init
 * Sec. 2: the initial graph gives every vertex k neighbours drawn uniformly at
 * random; the graph is simple, so the k ids are distinct and exclude the
 * vertex itself. Draw j = 0, 1, 2, ... maps H(seed,1,0,u,j) onto the N-1 other
 * ids by a multiply-high and skips repeats. All entries start NEW.
 */
int orc_init(const float *X, int64_t N, int32_t d, int32_t K, uint64_t seed,
             int32_t *ids, double *dists, uint8_t *flags)
{
    if (!X || !ids || !dists || !flags || N < 2 || d < 1 || K < 1 || K > N - 1)
        return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < N; ++u) {
        orc_entry *row = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)K);
        if (!row) { bad = 1; continue; }
        int32_t have = 0;
        for (uint32_t j = 0; have < K; ++j) {
            uint64_t h = orc_hash(seed, 1, 0, (uint32_t)u, j);
            uint64_t c = ((h >> 32) * (uint64_t)(N - 1)) >> 32;
            if ((int64_t)c >= u) c += 1;
            int dup = 0;
            for (int32_t i = 0; i < have; ++i)
                if (row[i].id == (int32_t)c) { dup = 1; break; }
            if (!dup) {
                row[have].id = (int32_t)c;
                row[have].dist = orc_dist(X, d, u, (int64_t)c);
                row[have].flag = ORC_NEW;
                ++have;
            }
        }
        qsort(row, (size_t)K, sizeof(orc_entry), cmp_entry);
        for (int32_t i = 0; i < K; ++i) {
            ids[u * K + i] = row[i].id;
            dists[u * K + i] = row[i].dist;
            flags[u * K + i] = row[i].flag;
        }
        free(row);
    }
    return bad ? -2 : 0;
}

/* ---------------------------------------------------------------- step 2: sample
 * Sec. 3.1: the neighbourhood of u is its forward list plus every w with u in
 * the list of w (reverse). Fused weighted sampling draws one uniform weight per
 * edge and keeps the rho*k smallest. Readings: the weight is keyed on the
 * unordered pair, w = H(seed,2,t,min,max) >> 32, so both routes to the same
 * member give the identical tuple (counted once); ties in w go to the smaller
 * member id; new and old pools are sampled separately with cap C each, and a
 * member sampled as new is removed from the old sample. Every forward NEW
 * entry whose target was sampled as new becomes OLD.
 *
 * Turbosampling (Sec. 3.1, mode ORC_TURBO): the heaps are replaced by a coin
 * per edge that keeps a member with probability rho*k/|N(u)|, |N(u)| being
 * the neighbourhood size the paper tracks on every graph update. Readings:
 * the coin is the same per-pair weight (kept iff w * n_f(u) < C * 2^32, exact
 * in integers), n_f(u) is the number of pool entries of flag f of u counted
 * with multiplicity (forward plus reverse, as the tracked size grows by one
 * per edge), so each flag keeps C members in expectation as the heap rule
 * does; the fixed neighbourhood bound is C per flag, and when more entries
 * than that pass, the C of smallest (w, id) stay. Everything else (duplicate
 * tuples, old members also sampled as new, the flip) is as in the heap rule,
 * so the turbo sample of each flag is a subset of the heap rule's.
 *
 * Outputs: cnew[u*C .. +nnew[u]) and cold[u*C .. +nold[u]) hold the sampled
 * member ids sorted by (w, id); flags_out holds the flags after the flip.
 */
typedef struct { uint32_t w; int32_t id; uint8_t flag; } orc_cand;

static int cmp_cand(const void *x, const void *y)
{
    const orc_cand *a = (const orc_cand *)x, *b = (const orc_cand *)y;
    if (a->flag != b->flag) return a->flag > b->flag ? -1 : 1; /* NEW first */
    if (a->w != b->w) return a->w < b->w ? -1 : 1;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return 0;
}

int orc_sample(const int32_t *ids, const uint8_t *flags_in, int64_t N, int32_t K,
               int32_t C, uint64_t seed, int32_t t,
               int32_t *cnew, int32_t *nnew, int32_t *cold, int32_t *nold,
               uint8_t *flags_out, int32_t mode)
{
    if (!ids || !flags_in || !cnew || !nnew || !cold || !nold || !flags_out ||
        N < 2 || K < 1 || C < 1 || C > K || (mode != ORC_WEIGHTED && mode != ORC_TURBO))
        return -1;
    /* reverse lists: rev(v) = {(u, flag of u->v)}, filled in ascending u */
    int64_t *roff = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int32_t *rsrc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N * K));
    uint8_t *rflg = (uint8_t *)malloc((size_t)(N * K));
    if (!roff || !rsrc || !rflg) { free(roff); free(rsrc); free(rflg); return -2; }
    for (int64_t e = 0; e < N * K; ++e) roff[ids[e] + 1] += 1;
    for (int64_t v = 0; v < N; ++v) roff[v + 1] += roff[v];
    {
        int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
        if (!cur) { free(roff); free(rsrc); free(rflg); return -2; }
        memcpy(cur, roff, sizeof(int64_t) * (size_t)N);
        for (int64_t u = 0; u < N; ++u)
            for (int32_t k = 0; k < K; ++k) {
                int32_t v = ids[u * K + k];
                rsrc[cur[v]] = (int32_t)u;
                rflg[cur[v]] = flags_in[u * K + k];
                cur[v] += 1;
            }
        free(cur);
    }
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < N; ++u) {
        int64_t P = K + (roff[u + 1] - roff[u]);
        orc_cand *pool = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)P);
        if (!pool) { bad = 1; continue; }
        int64_t n = 0;
        for (int32_t k = 0; k < K; ++k) {
            int32_t v = ids[u * K + k];
            uint32_t a = (uint32_t)(u < v ? u : v), b = (uint32_t)(u < v ? v : u);
            pool[n].w = (uint32_t)(orc_hash(seed, 2, (uint64_t)t, a, b) >> 32);
            pool[n].id = v;
            pool[n].flag = flags_in[u * K + k];
            ++n;
        }
        for (int64_t r = roff[u]; r < roff[u + 1]; ++r) {
            int32_t x = rsrc[r];
            uint32_t a = (uint32_t)(u < x ? u : x), b = (uint32_t)(u < x ? x : u);
            pool[n].w = (uint32_t)(orc_hash(seed, 2, (uint64_t)t, a, b) >> 32);
            pool[n].id = x;
            pool[n].flag = rflg[r];
            ++n;
        }
        qsort(pool, (size_t)n, sizeof(orc_cand), cmp_cand);
        uint64_t nf[2] = {0, 0}; /* pool entries per flag, with multiplicity */
        for (int64_t i = 0; i < n; ++i) nf[pool[i].flag == ORC_NEW ? 0 : 1] += 1;
        int32_t cn = 0, co_raw = 0;
        int32_t *old_raw = cold + u * C; /* first take the C smallest old, then drop members also in new */
        for (int64_t i = 0; i < n; ++i) {
            if (i > 0 && cmp_cand(&pool[i - 1], &pool[i]) == 0) continue; /* identical tuple */
            if (mode == ORC_TURBO &&
                (uint64_t)pool[i].w * nf[pool[i].flag == ORC_NEW ? 0 : 1] >= ((uint64_t)C << 32))
                continue; /* the coin dropped this edge */
            if (pool[i].flag == ORC_NEW) {
                if (cn < C) cnew[u * C + cn++] = pool[i].id;
            } else {
                if (co_raw < C) old_raw[co_raw++] = pool[i].id;
            }
        }
        int32_t co = 0;
        for (int32_t i = 0; i < co_raw; ++i) {
            int in_new = 0;
            for (int32_t j = 0; j < cn; ++j)
                if (cnew[u * C + j] == old_raw[i]) { in_new = 1; break; }
            if (!in_new) old_raw[co++] = old_raw[i];
        }
        nnew[u] = cn;
        nold[u] = co;
        for (int32_t k = 0; k < K; ++k) {
            uint8_t f = flags_in[u * K + k];
            if (f == ORC_NEW) {
                for (int32_t j = 0; j < cn; ++j)
                    if (cnew[u * C + j] == ids[u * K + k]) { f = ORC_OLD; break; }
            }
            flags_out[u * K + k] = f;
        }
        free(pool);
    }
    free(roff); free(rsrc); free(rflg);
    return bad ? -2 : 0;
}

/* ---------------------------------------------------------------- steps 3-4: join and merge
 * Sec. 2 (calculation step) and Fig. 1: evaluate the distances of the pairs
 * in each sampled neighbourhood and update G where a closer vertex was found.
 * Reading: pairs are new x new (unordered, p != q) and new x old; each pair
 * evaluated in owner u proposes q to p and p to q. The update is synchronous:
 * every proposal is judged against the lists as they were after sampling, and
 * the new list of p is the K smallest (distance, id) keys of its list and the
 * proposals whose id is not already in it. c_t counts ids that enter a list.
 */
typedef struct { int32_t target; int32_t src; double dist; } orc_prop;

int orc_join_merge(const float *X, int64_t N, int32_t d, int32_t K, int32_t C,
                   const int32_t *cnew, const int32_t *nnew,
                   const int32_t *cold, const int32_t *nold,
                   int32_t *ids, double *dists, uint8_t *flags,
                   int64_t *evals_out, int64_t *changes_out)
{
    if (!X || !cnew || !nnew || !cold || !nold || !ids || !dists || !flags ||
        N < 2 || d < 1 || K < 1 || C < 1)
        return -1;
    /* per-owner pair counts and proposal offsets (two proposals per pair) */
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)N + 1));
    if (!off) return -2;
    off[0] = 0;
    for (int64_t u = 0; u < N; ++u) {
        int64_t a = nnew[u], b = nold[u];
        int64_t pairs = a * (a - 1) / 2 + a * b;
        off[u + 1] = off[u] + 2 * pairs;
    }
    int64_t nprop = off[N];
    orc_prop *prop = (orc_prop *)malloc(sizeof(orc_prop) * (size_t)(nprop > 0 ? nprop : 1));
    if (!prop) { free(off); return -2; }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < N; ++u) {
        int64_t o = off[u];
        const int32_t *nw = cnew + u * C, *od = cold + u * C;
        for (int32_t i = 0; i < nnew[u]; ++i) {
            for (int32_t j = i + 1; j < nnew[u]; ++j) {
                double D = orc_dist(X, d, nw[i], nw[j]);
                prop[o++] = (orc_prop){nw[i], nw[j], D};
                prop[o++] = (orc_prop){nw[j], nw[i], D};
            }
            for (int32_t j = 0; j < nold[u]; ++j) {
                double D = orc_dist(X, d, nw[i], od[j]);
                prop[o++] = (orc_prop){nw[i], od[j], D};
                prop[o++] = (orc_prop){od[j], nw[i], D};
            }
        }
    }
    /* group proposals by target (stable counting sort) */
    int64_t *toff = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    orc_prop *byt = (orc_prop *)malloc(sizeof(orc_prop) * (size_t)(nprop > 0 ? nprop : 1));
    if (!toff || !byt) { free(off); free(prop); free(toff); free(byt); return -2; }
    for (int64_t i = 0; i < nprop; ++i) toff[prop[i].target + 1] += 1;
    for (int64_t v = 0; v < N; ++v) toff[v + 1] += toff[v];
    {
        int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
        if (!cur) { free(off); free(prop); free(toff); free(byt); return -2; }
        memcpy(cur, toff, sizeof(int64_t) * (size_t)N);
        for (int64_t i = 0; i < nprop; ++i) byt[cur[prop[i].target]++] = prop[i];
        free(cur);
    }
    free(prop);
    int64_t *chg = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < N; ++p) {
        int64_t q0 = toff[p], q1 = toff[p + 1];
        if (q0 == q1) continue;
        orc_entry *all = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)(K + (q1 - q0)));
        orc_entry *cand = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)(q1 - q0));
        if (!all || !cand) { free(all); free(cand); bad = 1; continue; }
        int64_t n = 0;
        for (int32_t k = 0; k < K; ++k)
            all[n++] = (orc_entry){dists[p * K + k], ids[p * K + k], flags[p * K + k]};
        /* candidates: each id once with its smallest key, and only ids that
         * are not already in the list (an existing entry keeps its flag) */
        for (int64_t i = q0; i < q1; ++i)
            cand[i - q0] = (orc_entry){byt[i].dist, byt[i].src, 2 /* marks a candidate */};
        qsort(cand, (size_t)(q1 - q0), sizeof(orc_entry), cmp_entry_by_id);
        for (int64_t i = 0; i < q1 - q0; ++i) {
            if (i > 0 && cand[i].id == cand[i - 1].id) continue;
            int in_list = 0;
            for (int32_t k = 0; k < K; ++k)
                if (all[k].id == cand[i].id) { in_list = 1; break; }
            if (!in_list) all[n++] = cand[i];
        }
        free(cand);
        qsort(all, (size_t)n, sizeof(orc_entry), cmp_entry);
        int64_t c = 0;
        for (int32_t k = 0; k < K; ++k) {
            uint8_t f = all[k].flag;
            if (f == 2) { f = ORC_NEW; ++c; }
            ids[p * K + k] = all[k].id;
            dists[p * K + k] = all[k].dist;
            flags[p * K + k] = f;
        }
        chg[p] = c;
        free(all);
    }
    int64_t changes = 0;
    for (int64_t p = 0; p < N; ++p) changes += chg[p];
    free(chg); free(byt); free(toff);
    if (evals_out) *evals_out = nprop / 2;
    if (changes_out) *changes_out = changes;
    free(off);
    return bad ? -2 : 0;
}

/* One full iteration t >= 1 (sample, then join and merge) on the state
 * (ids, dists, flags), updated in place. */
int orc_iterate(const float *X, int64_t N, int32_t d, int32_t K, int32_t C,
                uint64_t seed, int32_t t, int32_t *ids, double *dists, uint8_t *flags,
                int64_t *evals_out, int64_t *changes_out, int32_t mode)
{
    int32_t *cnew = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N * C));
    int32_t *cold = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N * C));
    int32_t *nnew = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *nold = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    uint8_t *f2 = (uint8_t *)malloc((size_t)(N * K));
    int rc = -2;
    if (cnew && cold && nnew && nold && f2) {
        rc = orc_sample(ids, flags, N, K, C, seed, t, cnew, nnew, cold, nold, f2, mode);
        if (rc == 0) {
            memcpy(flags, f2, (size_t)(N * K));
            rc = orc_join_merge(X, N, d, K, C, cnew, nnew, cold, nold, ids, dists, flags,
                                evals_out, changes_out);
        }
    }
    free(cnew); free(cold); free(nnew); free(nold); free(f2);
    return rc;
}

/* Block-asynchronous iteration t. The paper updates the graph in place
 * (Sec. 3.1 tracks neighbourhood sizes upon every update), so a node sampled
 * later in an iteration sees what earlier nodes changed. Reading (order-
 * dependent, so it is fixed here): the owners are taken in B blocks of
 * consecutive ids, block b = [floor(N b / B), floor(N (b + 1) / B)), in
 * order; block b samples from the graph as blocks 0..b-1 of this iteration
 * left it (lists, flags and the reverse lists they imply), only its owners
 * take samples, flip and join, and their proposals are merged into every
 * list before block b + 1 samples. B = 1 is the synchronous iteration and
 * B = N the node-by-node order. e_t and c_t are summed over the blocks (an
 * id that enters and is pushed out later in the iteration counts once). */
int orc_iterate_blocks(const float *X, int64_t N, int32_t d, int32_t K, int32_t C,
                       uint64_t seed, int32_t t, int32_t B, int32_t *ids, double *dists, uint8_t *flags,
                       int64_t *evals_out, int64_t *changes_out, int32_t mode)
{
    if (B < 1 || (int64_t)B > N) return -1;
    int32_t *cnew = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N * C));
    int32_t *cold = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N * C));
    int32_t *nnew = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *nold = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    uint8_t *f2 = (uint8_t *)malloc((size_t)(N * K));
    int rc = -2;
    int64_t e_sum = 0, c_sum = 0;
    if (cnew && cold && nnew && nold && f2) {
        rc = 0;
        for (int32_t b = 0; b < B && rc == 0; ++b) {
            const int64_t lo = N * (int64_t)b / B, hi = N * (int64_t)(b + 1) / B;
            rc = orc_sample(ids, flags, N, K, C, seed, t, cnew, nnew, cold, nold, f2, mode);
            if (rc != 0) break;
            for (int64_t u = 0; u < N; ++u) {
                if (u >= lo && u < hi) {
                    memcpy(flags + u * K, f2 + u * K, (size_t)K);
                } else {
                    nnew[u] = 0;
                    nold[u] = 0;
                }
            }
            int64_t e = 0, c = 0;
            rc = orc_join_merge(X, N, d, K, C, cnew, nnew, cold, nold, ids, dists, flags, &e, &c);
            e_sum += e;
            c_sum += c;
        }
    }
    free(cnew); free(cold); free(nnew); free(nold); free(f2);
    if (evals_out) *evals_out = e_sum;
    if (changes_out) *changes_out = c_sum;
    return rc;
}

/* Sum of all list distances, in a fixed order (the monotonicity invariant). */
double orc_dist_sum(const double *dists, int64_t N, int32_t K)
{
    double s = 0.0;
    for (int64_t i = 0; i < N * K; ++i) s += dists[i];
    return s;
}

/* Whole build (Sec. 2): init, then iterate until the number of changes falls
 * below delta*N*K (reading of the unspecified threshold) or max_iters is hit.
 * Per-iteration evals / changes / distance sums are written when the arrays
 * are given (capacity max_iters). Returns the number of iterations run. */
int orc_build(const float *X, int64_t N, int32_t d, int32_t K, double rho, double delta,
              int32_t max_iters, uint64_t seed, int32_t *ids, double *dists, uint8_t *flags,
              int64_t *evals, int64_t *changes, double *dsum, int32_t mode)
{
    if (rho <= 0.0 || rho > 1.0 || delta < 0.0 || max_iters < 0) return -1;
    int rc = orc_init(X, N, d, K, seed, ids, dists, flags);
    if (rc) return rc;
    int32_t C = orc_cap(K, rho);
    int32_t iters = 0;
    for (int32_t t = 1; t <= max_iters; ++t) {
        int64_t e = 0, c = 0;
        rc = orc_iterate(X, N, d, K, C, seed, t, ids, dists, flags, &e, &c, mode);
        if (rc) return rc;
        if (evals) evals[t - 1] = e;
        if (changes) changes[t - 1] = c;
        if (dsum) dsum[t - 1] = orc_dist_sum(dists, N, K);
        iters = t;
        if ((double)c < delta * (double)N * (double)K) break;
    }
    return iters;
}

/* ---------------------------------------------------------------- greedy reordering
 * Sec. 3.2 (greedy clustering heuristic): the memory order is grown one spot
 * at a time so that the node placed at spot i+1 is the nearest listed
 * neighbour of the node at spot i that has no spot yet. A host reference for
 * the device permutation's locality; it changes no list (the method's result
 * keeps original ids).
 * Readings: spot 0 holds node 0; a list is scanned nearest first (rows are
 * sorted by (D, id)); when every neighbour of the node at spot i is already
 * placed, spot i+1 takes the unplaced node of smallest id (the paper leaves
 * that spot to whatever its in-place exchanges put there).
 * Outputs: sigma[node] = spot and sigma_inv[spot] = node.
 */
int orc_greedy_order(const int32_t *ids, int64_t N, int32_t K, int32_t *sigma, int32_t *sigma_inv)
{
    if (!ids || !sigma || !sigma_inv || N < 1 || K < 1) return -1;
    uint8_t *placed = (uint8_t *)calloc((size_t)N, 1);
    if (!placed) return -2;
    int64_t lowest = 0;   /* every node below it has a spot */
    int32_t prev = 0;
    for (int64_t spot = 0; spot < N; ++spot) {
        int32_t node = -1;
        if (spot > 0) {
            const int32_t *nb = ids + (int64_t)prev * K;
            for (int32_t k = 0; k < K && node < 0; ++k)
                if (!placed[nb[k]]) node = nb[k];
        }
        if (node < 0) {
            while (placed[lowest]) ++lowest;
            node = (int32_t)lowest;
        }
        placed[node] = 1;
        sigma[node] = (int32_t)spot;
        sigma_inv[spot] = node;
        prev = node;
    }
    free(placed);
    return 0;
}

/* ---------------------------------------------------------------- exact K-NN
 * Sec. 2: the trivial K-NNG evaluates all n(n-1)/2 distances and keeps the k
 * best. Used for recall. Ties broken by id, like the lists above. */
int orc_bruteforce(const float *X, int64_t N, int32_t d, int32_t K, int32_t *ids, double *dists)
{
    if (!X || !ids || !dists || N < 2 || d < 1 || K < 1 || K > N - 1) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < N; ++p) {
        orc_entry *best = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)K);
        if (!best) { bad = 1; continue; }
        int32_t n = 0;
        for (int64_t q = 0; q < N; ++q) {
            if (q == p) continue;
            double D = orc_dist(X, d, p, q);
            if (n == K && !key_less(D, (int32_t)q, best[K - 1].dist, best[K - 1].id)) continue;
            int32_t i = n < K ? n++ : K - 1;
            while (i > 0 && key_less(D, (int32_t)q, best[i - 1].dist, best[i - 1].id)) {
                best[i] = best[i - 1];
                --i;
            }
            best[i] = (orc_entry){D, (int32_t)q, 0};
        }
        for (int32_t k = 0; k < K; ++k) {
            ids[p * K + k] = best[k].id;
            dists[p * K + k] = best[k].dist;
        }
        free(best);
    }
    return bad ? -2 : 0;
}

/* Exact K-NN for a subset of query rows (sampled recall at large N). */
int orc_bruteforce_rows(const float *X, int64_t N, int32_t d, int32_t K,
                        const int64_t *rows, int64_t nrows, int32_t *ids, double *dists)
{
    if (!X || !rows || !ids || !dists || N < 2 || d < 1 || K < 1 || K > N - 1) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t p = rows[r];
        orc_entry *best = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)K);
        if (!best) { bad = 1; continue; }
        int32_t n = 0;
        for (int64_t q = 0; q < N; ++q) {
            if (q == p) continue;
            double D = orc_dist(X, d, p, q);
            if (n == K && !key_less(D, (int32_t)q, best[K - 1].dist, best[K - 1].id)) continue;
            int32_t i = n < K ? n++ : K - 1;
            while (i > 0 && key_less(D, (int32_t)q, best[i - 1].dist, best[i - 1].id)) {
                best[i] = best[i - 1];
                --i;
            }
            best[i] = (orc_entry){D, (int32_t)q, 0};
        }
        for (int32_t k = 0; k < K; ++k) {
            ids[r * K + k] = best[k].id;
            dists[r * K + k] = best[k].dist;
        }
        free(best);
    }
    return bad ? -2 : 0;
}

/* D(p, ids[p][k]) for every list entry: checks stored distances and recall. */
int orc_list_dists(const float *X, int64_t N, int32_t d, int32_t K, const int32_t *ids, double *out)
{
    if (!X || !ids || !out) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p)
        for (int32_t k = 0; k < K; ++k)
            out[p * K + k] = orc_dist(X, d, p, ids[p * K + k]);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of later calls (results do not depend on it; timing only). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
