"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a published reference output,
a closed form, a textbook routine (numpy sort / brute force), an invariant of
the method, or a statistical property stated in the paper. Paper citations are
to Kluser et al., arXiv 2112.06630.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------- hash

def test_mix64_matches_splitmix64_reference_outputs(oracle_lib):
    """SplitMix64 (seed 0) reference outputs pin the mix64 output function."""
    vals = [int(l, 16) for l in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt"))
            if l.startswith("0x")]
    state = 0
    for v in vals:
        state = (state + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
        assert oracle.mix64(state) == v


def test_hash_weights_are_uniform(oracle_lib):
    """Sampling weights must be uniform in [0, 2^32) (Sec. 3.1 draws them u.a.r.):
    chi-square over 64 bins, and distinct (t, pair) inputs decorrelate."""
    w = np.array([oracle.hash64(7, 2, t, a, a + 1 + b) >> 32
                  for t in range(1, 5) for a in range(60) for b in range(60)], np.float64)
    hist, _ = np.histogram(w, bins=64, range=(0, 2.0**32))
    exp = len(w) / 64
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 120  # 63 dof, p ~ 1e-5
    assert len(np.unique(w)) == len(w)


def _unmix64(z):
    """Inverse of the SplitMix64 output function (pinned above): undo the
    xor-shifts and multiply by the inverses of the two odd constants mod 2^64."""
    M = 0xFFFFFFFFFFFFFFFF

    def unxorshift(y, s):
        x = y
        for _ in range(64 // s + 1):
            x = y ^ (x >> s)
        return x & M

    z = unxorshift(z, 31)
    z = (z * pow(0x94D049BB133111EB, -1, 1 << 64)) & M
    z = unxorshift(z, 27)
    z = (z * pow(0xBF58476D1CE4E5B9, -1, 1 << 64)) & M
    return unxorshift(z, 30)


def test_hash_composition_by_inverting_mix64(oracle_lib):
    """H(seed, tag, t, a, b) = mix64(mix64(mix64(seed + phi*(tag+1)) ^ t) ^ (a << 32 | b))
    (the counter-hash reading of Sec. 3.1's uniform weights and Sec. 2's random
    initial graph). mix64 is a bijection, so peeling one layer off with its
    inverse must expose (a << 32 | b) against H(., 0, 0), then t, then
    seed + phi*(tag+1); with seed 0 the innermost layer is the (tag+1)-th
    SplitMix64 output (the reference values)."""
    M = 0xFFFFFFFFFFFFFFFF
    PHI = 0x9E3779B97F4A7C15
    rng = np.random.default_rng(5)
    for z in rng.integers(0, 2**63, 20, dtype=np.int64).tolist():
        assert _unmix64(oracle.mix64(z)) == z
        assert _unmix64(oracle.mix64(z | (1 << 63))) == z | (1 << 63)
    for _ in range(40):
        seed = int(rng.integers(0, 2**63)) | (int(rng.integers(0, 2)) << 63)
        tag = int(rng.integers(1, 3))
        t = int(rng.integers(0, 1000))
        a, b = (int(x) for x in rng.integers(0, 2**31, 2))
        h = oracle.hash64(seed, tag, t, a, b)
        inner = _unmix64(oracle.hash64(seed, tag, t, 0, 0))
        assert _unmix64(h) ^ inner == (a << 32) | b
        assert _unmix64(inner) ^ _unmix64(_unmix64(oracle.hash64(seed, tag, 0, 0, 0))) == t
        assert _unmix64(_unmix64(_unmix64(oracle.hash64(seed, tag, 0, 0, 0)))) == (seed + PHI * (tag + 1)) & M
    vals = [int(l, 16) for l in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt")) if l.startswith("0x")]
    for tag in (0, 1):
        assert _unmix64(_unmix64(oracle.hash64(0, tag, 0, 0, 0))) == vals[tag]


@pytest.mark.parametrize("K,rho,C", [(15, 0.5, 8), (20, 0.5, 10), (20, 1.0, 20), (9, 0.3, 3), (10, 0.25, 3),
                                     (10, 0.01, 1), (1, 1.0, 1), (64, 1.0, 64), (7, 0.9, 7)])
def test_cap_closed_forms(oracle_lib, K, rho, C):
    """C = min(K, max(1, ceil(rho*K))): Sec. 3.1 samples rho*k per neighbourhood;
    a non-integer rho*k is rounded up (15 * 0.5 = 7.5 -> 8, 9 * 0.3 = 2.7 -> 3),
    and at least one member is sampled (10 * 0.01 -> 1)."""
    assert oracle.cap(K, rho) == C


# --------------------------------------------------------------------------- distances / brute force

def test_dist_matches_numpy_on_integer_points(oracle_lib):
    X = synth.integer_points(50, 7, 30, 1)
    ids = np.tile(np.arange(50, dtype=np.int32), (50, 1))
    D = oracle.list_dists(X, ids)
    ref = ((X.astype(np.float64)[:, None, :] - X.astype(np.float64)[None, :, :]) ** 2).sum(-1)
    assert np.array_equal(D, ref)


@pytest.mark.parametrize("N,d,K,seed", [(60, 3, 5, 0), (100, 8, 10, 1), (37, 1, 36, 2)])
def test_bruteforce_matches_numpy_lexsort(oracle_lib, N, d, K, seed):
    """Sec. 2: the exact K-NNG keeps the k nearest others; (dist, id) tie-break.
    Integer data makes ties frequent, so the tie-break is exercised."""
    X = synth.integer_points(N, d, 4, seed)
    ids, dists = oracle.bruteforce(X, K)
    Xd = X.astype(np.float64)
    D = ((Xd[:, None, :] - Xd[None, :, :]) ** 2).sum(-1)
    for p in range(N):
        order = np.lexsort((np.arange(N), D[p]))
        order = order[order != p][:K]
        assert np.array_equal(ids[p], order)
        assert np.array_equal(dists[p], D[p, order])


# --------------------------------------------------------------------------- init

def test_init_rows_are_distinct_nonself_sorted(oracle_lib):
    X = synth.integer_points(300, 4, 5, 3)
    st = oracle.init(X, 12, 99)
    D = oracle.list_dists(X, st.ids)
    for u in range(300):
        row = st.ids[u]
        assert len(set(row.tolist())) == 12 and u not in row
        keys = list(zip(st.dists[u], row))
        assert keys == sorted(keys)
    assert np.array_equal(D, st.dists)
    assert (st.flags == oracle.NEW).all()


def test_init_complete_graph_when_N_is_K_plus_1(oracle_lib):
    """N = K + 1 leaves no choice: every list holds all other points, in (dist, id) order."""
    X = synth.integer_points(11, 2, 3, 5)
    st = oracle.init(X, 10, 1234)
    ids, dists = oracle.bruteforce(X, 10)
    assert np.array_equal(st.ids, ids) and np.array_equal(st.dists, dists)


def test_init_ids_uniform(oracle_lib):
    """Sec. 2: initial neighbours are drawn uniformly from V (chi-square on frequencies)."""
    N, K = 400, 10
    X = np.zeros((N, 1), np.float32)
    cnt = np.zeros(N)
    for s in range(10):
        st = oracle.init(X, K, s)
        np.add.at(cnt, st.ids.reshape(-1), 1)
    exp = cnt.sum() / N
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < N + 5 * math.sqrt(2 * N)


def test_init_cluster_miss_rate_bound(oracle_lib):
    """Sec. 3.2: Pr[none of k random neighbours in the own cluster] <= ((c-1)/c)^k.
    Sampling without replacement makes the rate slightly lower than the bound."""
    N, K, c = 4000, 10, 10
    X, lab = synth.clustered_labels(N, 4, c, 11)
    st = oracle.init(X, K, 5)
    miss = np.mean([(lab[st.ids[u]] != lab[u]).all() for u in range(N)])
    bound = ((c - 1) / c) ** K
    assert miss <= bound + 3 * math.sqrt(bound * (1 - bound) / N)
    assert miss >= 0.75 * bound


# --------------------------------------------------------------------------- sample

def _rev(st):
    N = st.ids.shape[0]
    rev = [set() for _ in range(N)]
    for u in range(N):
        for v in st.ids[u]:
            rev[v].add(u)
    return rev


def test_sample_bounds_and_membership(oracle_lib):
    """Sec. 3.1: N(u) draws from forward and reverse neighbours, bounded by rho*k per flag."""
    X, p = synth.workload("gauss2k_d8", N=600)
    K, C = 10, oracle.cap(10, 0.5)
    r = oracle.build_graph(X, K, 0.5, 0.0, 2, 3)
    st = oracle.State(r.ids, r.dists, r.flags, 2)
    sm = oracle.sample(st, K, C, 3, 3)
    rev = _rev(st)
    for u in range(600):
        nw, od = set(sm.cnew[u].tolist()), set(sm.cold[u].tolist())
        assert len(nw) == len(sm.cnew[u]) <= C and len(od) == len(sm.cold[u]) <= C
        assert not (nw & od)
        assert (nw | od) <= (set(st.ids[u].tolist()) | rev[u])
        assert u not in nw | od


def test_sample_complete_graph_selects_everyone_and_flips(oracle_lib):
    """N = K + 1 with C = K: the pool is every other point (forward and reverse
    routes give the identical tuple, counted once), so all are sampled new, all
    forward entries flip to OLD, e_1 = N*K(K-1)/2, nothing changes, and a second
    iteration has no new member left (e_2 = 0)."""
    N, K = 9, 8
    X = synth.integer_points(N, 3, 10, 2)
    st = oracle.init(X, K, 4)
    sm = oracle.sample(st, K, K, 4, 1)
    for u in range(N):
        assert sorted(sm.cnew[u].tolist()) == [v for v in range(N) if v != u]
        assert len(sm.cold[u]) == 0
    assert (sm.flags == oracle.OLD).all()
    s1, e1, c1 = oracle.iterate(X, st, K, K, 4)
    assert e1 == N * K * (K - 1) // 2 and c1 == 0
    assert np.array_equal(s1.ids, st.ids)
    s2, e2, c2 = oracle.iterate(X, s1, K, K, 4)
    assert e2 == 0 and c2 == 0


def test_sample_selection_is_uniform(oracle_lib):
    """Sec. 3.1: keeping the rho*k smallest u.a.r. weights is a uniform subset.
    Over many iterations t (fresh weights), every pool member of a fixed node is
    chosen with frequency C/|pool|."""
    N, K, C = 200, 10, 3
    X = np.zeros((N, 1), np.float32)
    st = oracle.init(X, K, 21)
    rev = _rev(st)
    T = 400
    counts = [dict() for _ in range(N)]
    for t in range(1, T + 1):
        sm = oracle.sample(st, K, C, 21, t)
        for u in range(0, N, 10):
            for v in sm.cnew[u]:
                counts[u][int(v)] = counts[u].get(int(v), 0) + 1
    chi2, dof = 0.0, 0
    for u in range(0, N, 10):
        pool = set(st.ids[u].tolist()) | rev[u]
        exp = T * C / len(pool)
        for v in pool:
            chi2 += (counts[u].get(v, 0) - exp) ** 2 / exp
            dof += 1
        assert set(counts[u]) <= pool
    assert chi2 < dof + 5 * math.sqrt(2 * dof)


def test_evals_count_closed_form(oracle_lib):
    """e_t = sum_u [n_new(n_new-1)/2 + n_new*n_old] (new x new and new x old pairs)."""
    X, _ = synth.workload("gauss2k_d8", N=500)
    K, C = 10, 7
    st = oracle.init(X, K, 8)
    sm = oracle.sample(st, K, C, 8, 1)
    exp = sum(len(a) * (len(a) - 1) // 2 + len(a) * len(b) for a, b in zip(sm.cnew, sm.cold))
    _, e, _ = oracle.iterate(X, st, K, C, 8)
    assert e == exp


# --------------------------------------------------------------------------- turbosampling

def _random_state(N, K, seed, p_new=0.5):
    """A random graph (distinct non-self members per row) with random flags."""
    rng = np.random.default_rng(seed)
    ids = np.empty((N, K), np.int32)
    for u in range(N):
        c = rng.choice(N - 1, K, replace=False)
        ids[u] = np.where(c >= u, c + 1, c)
    flags = np.where(rng.random((N, K)) < p_new, oracle.NEW, oracle.OLD).astype(np.uint8)
    return oracle.State(ids, np.zeros((N, K)), flags, 0)


def _turbo_by_definition(st, C, seed, t):
    """Sec. 3.1 turbosampling spelled out on one owner at a time: every edge
    (forward and reverse) is a pool entry with the pair's weight; entry of flag
    f survives when w * n_f < C * 2^32 (n_f: entries of flag f); identical
    (w, id, flag) entries count once; the C smallest (w, id) survivors per flag
    are kept; old members also kept as new are dropped."""
    N, K = st.ids.shape
    pools = [[] for _ in range(N)]
    for u in range(N):
        for k in range(K):
            v = int(st.ids[u, k])
            f = int(st.flags[u, k])
            w = oracle.hash64(seed, 2, t, min(u, v), max(u, v)) >> 32
            pools[u].append((w, v, f))
            pools[v].append((w, u, f))
    out = []
    for u in range(N):
        n = {f: sum(1 for e in pools[u] if e[2] == f) for f in (oracle.NEW, oracle.OLD)}
        keep = sorted({e for e in pools[u] if e[0] * n[e[2]] < (C << 32)})
        nw = [e[1] for e in keep if e[2] == oracle.NEW][:C]
        od = [e[1] for e in keep if e[2] == oracle.OLD][:C]
        out.append((nw, [x for x in od if x not in nw]))
    return out


@pytest.mark.parametrize("N,K,rho,seed,t", [(30, 5, 1.0, 1, 1), (40, 6, 0.5, 2, 3), (25, 8, 0.25, 3, 7)])
def test_turbo_matches_definition_by_brute_force(oracle_lib, N, K, rho, seed, t):
    """Brute force on tiny random states (mixed flags, mutual pairs present)."""
    st = _random_state(N, K, seed)
    C = oracle.cap(K, rho)
    sm = oracle.sample(st, K, C, seed, t, sampling="turbo")
    exp = _turbo_by_definition(st, C, seed, t)
    for u in range(N):
        assert sm.cnew[u].tolist() == exp[u][0]
        assert sm.cold[u].tolist() == exp[u][1]
        for k in range(K):
            f = st.flags[u, k]
            if f == oracle.NEW and int(st.ids[u, k]) in exp[u][0]:
                f = oracle.OLD
            assert sm.flags[u, k] == f


def test_turbo_equals_heap_rule_when_pools_are_small(oracle_lib):
    """With n_f <= C the coin keeps every entry (probability 1), so owners
    whose pools of both flags are that small sample exactly as the heap rule."""
    N, K, C = 400, 6, 6
    st = _random_state(N, K, 11, p_new=0.5)
    rev = [[0, 0] for _ in range(N)]
    for u in range(N):
        for k in range(K):
            rev[u][int(st.flags[u, k] == oracle.NEW)] += 1
            rev[int(st.ids[u, k])][int(st.flags[u, k] == oracle.NEW)] += 1
    small = [u for u in range(N) if max(rev[u]) <= C]
    assert len(small) > 20
    a = oracle.sample(st, K, C, 11, 2, sampling="turbo")
    b = oracle.sample(st, K, C, 11, 2, sampling="weighted")
    for u in small:
        assert a.cnew[u].tolist() == b.cnew[u].tolist()
        assert a.cold[u].tolist() == b.cold[u].tolist()
        assert np.array_equal(a.flags[u], b.flags[u])


def test_turbo_kept_counts_follow_the_coin(oracle_lib):
    """Each entry of flag f passes with probability C/n_f (Sec. 3.1), so on a
    random graph (mutual pairs rare) the kept count of flag f is
    min(C, Binomial(n_f, C/n_f)). The total over owners must match the sum of
    those expectations within 6 standard deviations; counting the whole pool
    instead of the flag's entries, or skipping the coin, moves it far out."""
    from scipy.stats import binom
    N, K, rho = 6000, 10, 0.5
    C = oracle.cap(K, rho)
    st = _random_state(N, K, 5, p_new=0.7)
    n = np.zeros((N, 2), np.int64)
    for u in range(N):
        for k in range(K):
            j = 1 if st.flags[u, k] == oracle.NEW else 0
            n[u, j] += 1
            n[int(st.ids[u, k]), j] += 1
    sm = oracle.sample(st, K, C, 5, 4, sampling="turbo")
    for j, got in ((1, sum(len(a) for a in sm.cnew)), (0, sum(len(a) for a in sm.cold))):
        mean = var = 0.0
        for m in n[:, j]:
            if m == 0:
                continue
            p = min(1.0, C / m)
            x = np.arange(0, m + 1)
            pm = binom.pmf(x, m, p)
            y = np.minimum(x, C)
            mu = float((pm * y).sum())
            mean += mu
            var += float((pm * (y - mu) ** 2).sum())
        assert abs(got - mean) < 6 * math.sqrt(var) + 0.002 * mean, (got, mean, math.sqrt(var))
    assert sum(len(a) for a in sm.cnew) < sum(min(C, m) for m in n[:, 1])


def test_turbo_new_sample_is_within_heap_sample(oracle_lib):
    """The coin only removes entries from the heap rule's ordering, so per owner
    the turbo new sample is a prefix of the heap rule's new sample, and at t = 1
    (every flag NEW) e_1 cannot exceed the heap rule's."""
    X, _ = synth.workload("gauss2k_d8", N=800)
    K, C = 10, oracle.cap(10, 1.0)
    st = oracle.init(X, K, 9)
    a = oracle.sample(st, K, C, 9, 1, sampling="turbo")
    b = oracle.sample(st, K, C, 9, 1, sampling="weighted")
    for u in range(800):
        assert b.cnew[u].tolist()[:len(a.cnew[u])] == a.cnew[u].tolist()
    _, ea, _ = oracle.iterate(X, st, K, C, 9, "turbo")
    _, eb, _ = oracle.iterate(X, st, K, C, 9, "weighted")
    assert ea < eb


def test_turbo_build_converges(oracle_lib):
    """A turbosampled build still finds most exact neighbours (recall vs brute force)."""
    X, _ = synth.workload("gauss2k_d8", N=1500)
    K = 10
    r = oracle.build_graph_c(X, K, 1.0, 0.001, 30, 4, sampling="turbo")
    ids, _ = oracle.bruteforce(X, K)
    rec = np.mean([len(set(r.ids[u]) & set(ids[u])) / K for u in range(1500)])
    assert r.iters < 30 and rec > 0.9


# --------------------------------------------------------------------------- greedy reordering (Alg. 1)

def _window_purity(labels, w, stride):
    n_lab = int(labels.max()) + 1
    return np.array([np.bincount(labels[s:s + w], minlength=n_lab).max() / w
                     for s in range(0, len(labels) - w + 1, stride)])


def test_greedy_order_is_a_permutation_with_its_inverse(oracle_lib):
    X, _ = synth.workload("gauss2k_d8", N=1500)
    r = oracle.build_graph(X, 10, 1.0, 0.0, 1, 2)
    sig, inv = oracle.greedy_order(r.ids)
    assert sorted(sig.tolist()) == list(range(1500))
    assert np.array_equal(inv[sig], np.arange(1500))
    assert np.array_equal(sig[inv], np.arange(1500))


def test_greedy_order_places_the_nearest_unplaced_neighbour_next(oracle_lib):
    """Sec. 3.2: spots up to i never change after step i - 1, so in the final
    order the node at spot i + 1 is the first entry of the (nearest-first) list
    of the node at spot i that does not sit at a spot <= i, whenever there is
    one; otherwise the step leaves spot i + 1 alone."""
    X, _ = synth.workload("gauss2k_d8", N=1200)
    r = oracle.build_graph(X, 8, 1.0, 0.0, 2, 4)
    sig, inv = oracle.greedy_order(r.ids)
    constrained = 0
    for i in range(1199):
        cand = [int(a) for a in r.ids[inv[i]] if sig[a] > i]
        if cand:
            assert inv[i + 1] == cand[0], i
            constrained += 1
    assert constrained > 600


def test_greedy_order_recovers_clusters_first(oracle_lib):
    """Sec. 4 (Fig. 4): on clustered data (n = 16384, d = 8, 8 clusters) the
    order built from G_1 keeps long single-cluster runs at the start, where
    many nodes are unplaced, and mixes towards 1/8 at the end."""
    X, lab = synth.gaussian_mixture(16384, 8, 8, 3, return_labels=True)
    st = oracle.init(X, 20, 3)
    s1, _, _ = oracle.iterate(X, st, 20, 20, 3)
    sig, inv = oracle.greedy_order(s1.ids)
    pur = _window_purity(lab[inv], 2000, 1024)
    base = _window_purity(lab, 2000, 1024).mean()
    assert base < 0.2
    assert pur[:8].mean() > 3 * base
    assert pur[-2:].mean() < 0.25


# --------------------------------------------------------------------------- join + merge

def _sorted_random_state(X, K, seed, p_new=0.6):
    """A random graph with the true distances (integer data: exact), rows sorted
    by (D, id), random NEW/OLD flags."""
    N = X.shape[0]
    st = _random_state(N, K, seed, p_new)
    Xi = X.astype(np.int64)
    for u in range(N):
        dd = ((Xi[st.ids[u]] - Xi[u]) ** 2).sum(1)
        order = np.lexsort((st.ids[u], dd))
        st.ids[u] = st.ids[u][order]
        st.flags[u] = st.flags[u][order]
        st.dists[u] = dd[order].astype(np.float64)
    return st


def _join_merge_by_definition(X, st, smp, K):
    """Sec. 2's calculation step written out per pair: in each owner's sample,
    every new x new pair (p != q, unordered) and every new x old pair is
    evaluated once and proposes each of its two points to the other; the new
    list of p is the K smallest (D, id) of its list and of the proposed ids not
    already in it (each such id once); ids that enter are NEW, kept entries keep
    the flag they have after sampling; c_t counts the ids that entered."""
    N = X.shape[0]
    Xi = X.astype(np.int64)
    props = [dict() for _ in range(N)]
    e = 0
    for u in range(N):
        nw = [int(x) for x in smp.cnew[u]]
        od = [int(x) for x in smp.cold[u]]
        pairs = [(nw[i], nw[j]) for i in range(len(nw)) for j in range(i + 1, len(nw))]
        pairs += [(a, b) for a in nw for b in od]
        e += len(pairs)
        for a, b in pairs:
            dd = float(((Xi[a] - Xi[b]) ** 2).sum())
            props[a][b] = dd
            props[b][a] = dd
    ids, dists, flags = st.ids.copy(), st.dists.copy(), smp.flags.copy()
    c = 0
    for p in range(N):
        listed = set(st.ids[p].tolist())
        ent = [(float(st.dists[p, k]), int(st.ids[p, k]), int(smp.flags[p, k]), 0) for k in range(K)]
        ent += [(dd, q, oracle.NEW, 1) for q, dd in props[p].items() if q not in listed]
        ent.sort(key=lambda x: (x[0], x[1]))
        for k, (dd, q, f, fresh) in enumerate(ent[:K]):
            ids[p, k], dists[p, k], flags[p, k] = q, dd, f
            c += fresh
    return ids, dists, flags, e, c


@pytest.mark.parametrize("N,K,rho,seed,t", [(40, 5, 1.0, 1, 1), (60, 6, 0.5, 2, 2), (50, 8, 0.75, 3, 4),
                                             (30, 4, 0.25, 4, 1)])
def test_join_merge_matches_definition_by_brute_force(oracle_lib, N, K, rho, seed, t):
    """One join + merge of the oracle equals the step written out pair by pair,
    on random states with mixed flags and small integer coordinates (exact
    distances, frequent ties: the (D, id) order decides)."""
    X = synth.integer_points(N, 3, 4, seed)
    st = _sorted_random_state(X, K, seed)
    C = oracle.cap(K, rho)
    smp = oracle.sample(st, K, C, seed, t)
    got, e, c = oracle.join_merge(X, st, smp, K, C)
    ids, dists, flags, e_ref, c_ref = _join_merge_by_definition(X, st, smp, K)
    assert e == e_ref and c == c_ref and c > 0
    assert np.array_equal(got.ids, ids)
    assert np.array_equal(got.dists, dists)
    assert np.array_equal(got.flags, flags)


def test_exact_knn_is_a_fixed_point(oracle_lib):
    """Feeding the exact K-NNG (all NEW) changes nothing: no proposal can beat it."""
    X, _ = synth.workload("gauss2k_d8", N=400)
    K = 10
    ids, dists = oracle.bruteforce(X, K)
    st = oracle.State(ids, dists, np.ones_like(ids, dtype=np.uint8), 0)
    s1, e, c = oracle.iterate(X, st, K, K, 5)
    assert c == 0 and e > 0
    assert np.array_equal(s1.ids, ids) and np.array_equal(s1.dists, dists)


def test_iteration_invariants_and_monotone_keys(oracle_lib):
    """Rows: K distinct non-self ids sorted by (dist, id), stored D = recomputed D;
    the i-th key of every row never increases, so sum of list distances never increases."""
    X, p = synth.workload("gauss2k_d8", N=800)
    K, C = 10, 10
    st = oracle.init(X, K, 2)
    prev_sum = st.dists.sum()
    for t in range(1, 7):
        nxt, e, c = oracle.iterate(X, st, K, C, 2)
        assert np.array_equal(oracle.list_dists(X, nxt.ids), nxt.dists)
        for u in range(800):
            assert len(set(nxt.ids[u].tolist())) == K and u not in nxt.ids[u]
            keys = list(zip(nxt.dists[u], nxt.ids[u]))
            assert keys == sorted(keys)
            old = list(zip(st.dists[u], st.ids[u]))
            assert all(a <= b for a, b in zip(keys, old))
        s = nxt.dists.sum()
        assert s <= prev_sum
        changed = sum(len(set(nxt.ids[u]) - set(st.ids[u])) for u in range(800))
        assert changed == c
        prev_sum, st = s, nxt


def test_build_reaches_exact_knn_on_small_inputs(oracle_lib):
    """Sec. 2: NN-Descent approximates the exact K-NNG; the paper reports recall
    above 99% (Sec. 2). On small clustered inputs the oracle must get there."""
    X, p = synth.workload("gauss2k_d8")
    r = oracle.build_graph(X, p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"])
    ei, ed = oracle.bruteforce(X, p["K"])
    assert oracle.recall(X, r.ids, ed) >= 0.99
    assert oracle.plain_recall(r.ids, ei) >= 0.99
    assert r.changes[-1] < p["delta"] * X.shape[0] * p["K"] or r.iters == p["max_iters"]


def test_identical_points_pure_id_tiebreak(oracle_lib):
    """All points equal: every distance is 0 and only ids order the lists."""
    N, K = 40, 6
    X = np.full((N, 3), 2.5, np.float32)
    r = oracle.build_graph(X, K, 1.0, 0.0, 15, 3)
    for u in range(N):
        assert (r.dists[u] == 0).all()
        assert list(r.ids[u]) == sorted(r.ids[u])
    exact = np.array([[v for v in range(N) if v != u][:K] for u in range(N)])
    assert oracle.plain_recall(r.ids, exact) >= 0.95


def test_stop_rule(oracle_lib):
    """Sec. 2: iterate until the number of changes falls below the threshold."""
    X, p = synth.workload("gauss2k_d8", N=1000)
    r = oracle.build_graph(X, 10, 1.0, 0.01, 50, 0)
    thr = 0.01 * 1000 * 10
    assert r.changes[-1] < thr and (r.changes[:-1] >= thr).all()
    r0 = oracle.build_graph(X, 10, 1.0, 0.01, 0, 0)
    assert r0.iters == 0


def test_c_build_equals_stepwise_build(oracle_lib):
    X, p = synth.workload("gauss2k_d8", N=700)
    a = oracle.build_graph(X, 10, 0.7, 0.001, 12, 9)
    b = oracle.build_graph_c(X, 10, 0.7, 0.001, 12, 9)
    assert a.iters == b.iters
    assert np.array_equal(a.ids, b.ids) and np.array_equal(a.dists, b.dists)
    assert np.array_equal(a.evals, b.evals) and np.array_equal(a.changes, b.changes)


def test_thread_count_independence(oracle_lib):
    """Results must not depend on the OpenMP thread count."""
    code = ("import numpy as np, oracle, synth, sys\n"
            "X,p=synth.workload('gauss2k_d8', N=900)\n"
            "r=oracle.build_graph_c(X,10,0.8,0.001,10,4)\n"
            "sys.stdout.write(str(hash(r.ids.tobytes()+r.dists.tobytes()+r.evals.tobytes())))\n")
    outs = []
    for n in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=n, PYTHONHASHSEED="0")
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env,
                                            cwd=os.path.dirname(HERE)))
    assert outs[0] == outs[1]


def _blocks_by_definition(X, st, K, C, seed, t, B):
    """The block-asynchronous iteration composed from its definition: block b
    of consecutive owner ids samples from the graph the earlier blocks left
    (the oracle's sampler, pinned above), only its owners keep their samples
    and flips, and its join + merge is the pair-by-pair step written out
    above."""
    N = X.shape[0]
    cur = st.copy()
    e_sum = c_sum = 0
    for b in range(B):
        lo, hi = N * b // B, N * (b + 1) // B
        smp = oracle.sample(cur, K, C, seed, t)
        for u in range(N):
            if not lo <= u < hi:
                smp.cnew[u] = smp.cnew[u][:0]
                smp.cold[u] = smp.cold[u][:0]
                smp.flags[u] = cur.flags[u]
        ids, dists, flags, e, c = _join_merge_by_definition(X, cur, smp, K)
        cur = oracle.State(ids, dists, flags, cur.t)
        e_sum += e
        c_sum += c
    return cur, e_sum, c_sum


@pytest.mark.parametrize("N,K,rho,seed,t,B", [(40, 5, 1.0, 1, 1, 4), (60, 6, 0.5, 2, 2, 3), (30, 4, 1.0, 4, 1, 30)])
def test_block_async_matches_definition(oracle_lib, N, K, rho, seed, t, B):
    """The block-asynchronous iteration (the paper's in-place update at block
    granularity, B = N: node by node) equals its definition composed block by
    block, on random states with exact integer distances."""
    X = synth.integer_points(N, 3, 4, seed)
    st = _sorted_random_state(X, K, seed)
    st.t = t - 1
    C = oracle.cap(K, rho)
    got, e, c = oracle.iterate(X, st, K, C, seed, blocks=B)
    ref, e_ref, c_ref = _blocks_by_definition(X, st, K, C, seed, t, B)
    assert e == e_ref and c == c_ref
    assert np.array_equal(got.ids, ref.ids)
    assert np.array_equal(got.dists, ref.dists)
    assert np.array_equal(got.flags, ref.flags)


def test_block_async_one_block_is_synchronous_and_more_blocks_differ(oracle_lib):
    """B = 1 is the synchronous iteration bit for bit; with several blocks the
    later blocks see the earlier ones' updates, so the trajectory changes, and
    the built graph stays valid and as good (recall against brute force)."""
    X, p = synth.workload("gauss2k_d8", N=800)
    K, C = 10, oracle.cap(10, 1.0)
    s0 = oracle.init(X, K, 0)
    a, ea, ca = oracle.iterate(X, s0, K, C, 0)
    b, eb, cb = oracle.iterate(X, s0, K, C, 0, blocks=1)
    assert np.array_equal(a.ids, b.ids) and np.array_equal(a.flags, b.flags) and (ea, ca) == (eb, cb)
    g, eg, cg = oracle.iterate(X, s0, K, C, 0, blocks=8)
    assert not np.array_equal(g.ids, a.ids)
    r = oracle.build_graph(X, K, 1.0, 0.001, 20, 0, blocks=8)
    s = oracle.build_graph(X, K, 1.0, 0.001, 20, 0)
    _, ed = oracle.bruteforce(X, K)
    assert oracle.recall(X, r.ids, ed) >= min(0.98, oracle.recall(X, s.ids, ed) - 0.01)
    assert (np.diff(r.dists, axis=1) >= 0).all()
