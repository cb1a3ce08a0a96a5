"""Turbosampling (Sec. 3.1: a Bernoulli coin of probability rho*k/|N(u)| in
place of the bounded heaps) on the GPU against the FP64 oracle's turbo rule.

Sampled sets along an oracle trajectory; one iteration on loaded graphs whose
hub members give pools of every select form (two owners per wave, one owner
per wave, the threshold select with the LDS cache and without it); whole
builds bit for bit on integer data for every join path; the batched form; and
the benchmark workload at full size.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def knng():
    import paper_2112_06630_amd as k
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return k


def dev(X):
    return torch.from_numpy(np.ascontiguousarray(X, np.float32)).to("cuda:0")


@pytest.mark.parametrize("rho", [1.0, 0.5, 0.25])
def test_turbo_sample_sets_match_oracle(knng, rho):
    """Sampled new/old sets are integer-exact for every t of an oracle trajectory."""
    X, _ = synth.workload("gauss2k_d8", N=1500)
    K = 10
    C = oracle.cap(K, rho)
    r = oracle.build_graph(X, K, rho, 0.0, 5, 7, keep_states=True, sampling="turbo")
    for s in r.states[:-1]:
        ctx = knng.Context(dev(X), K, rho=rho, seed=7, sampling="turbo")
        ctx.load(torch.from_numpy(s.ids), torch.from_numpy(s.flags), s.t)
        ctx.iterate()
        nw, od, cnt = (a.cpu().numpy() for a in ctx.samples())
        sm = oracle.sample(s, K, C, 7, s.t + 1, sampling="turbo")
        for u in range(X.shape[0]):
            a, b = cnt[u]
            assert list(nw[u, :a]) == list(sm.cnew[u]), (s.t, u)
            assert list(od[u, :b]) == list(sm.cold[u]), (s.t, u)
        ctx.close()


def hub_state(X, K, seed, hubs, t):
    """A graph whose rows list the hub members (id, fraction of rows) first and
    random other points after; random flags; rows sorted by (distance, id)."""
    N = X.shape[0]
    rng = np.random.default_rng(seed)
    ids = np.empty((N, K), np.int32)
    for u in range(N):
        row = [h for h, frac in hubs if h != u and rng.random() < frac]
        for c in rng.permutation(N):
            if len(row) == K:
                break
            if c != u and c not in row:
                row.append(int(c))
        ids[u] = row
    flags = np.where(rng.random((N, K)) < 0.6, oracle.NEW, oracle.OLD).astype(np.uint8)
    D = oracle.list_dists(X, ids)
    o = np.lexsort((ids, D))
    take = lambda a: np.take_along_axis(a, o, axis=1)
    return oracle.State(take(ids), take(D), take(flags), t)


# pools: hub 0 ~ 0.75 N + K entries (threshold select, weights read again),
# hub 1 ~ 0.3 N + K (threshold select from the LDS cache), hub 2 ~ 0.04 N + K
# (one owner per wave), everyone else <= 32 (two owners per wave)
HUBS = [(0, 0.75), (1, 0.3), (2, 0.04)]


# C <= 30: the threshold select for pools beyond 64 entries; C > 30 (K = 40,
# and K = 64 at rho = 0.5): the rank-based select of k_select_large
@pytest.mark.parametrize("K,rho", [(10, 1.0), (16, 1.0), (20, 0.5), (30, 1.0), (40, 1.0), (64, 0.5)])
@pytest.mark.parametrize("sampling", ["weighted", "turbo"])
def test_hub_pools_one_iteration(knng, K, rho, sampling):
    N = 900
    X = synth.integer_points(N, 8, 12, 3)
    s = hub_state(X, K, 5, HUBS, 2)
    C = oracle.cap(K, rho)
    ctx = knng.Context(dev(X), K, rho=rho, seed=9, path="valu", sampling=sampling)
    ctx.load(torch.from_numpy(s.ids), torch.from_numpy(s.flags), s.t)
    e, c = ctx.iterate()
    nw, od, cnt = (a.cpu().numpy() for a in ctx.samples())
    sm = oracle.sample(s, K, C, 9, s.t + 1, sampling=sampling)
    for u in range(N):
        a, b = cnt[u]
        assert list(nw[u, :a]) == list(sm.cnew[u]), u
        assert list(od[u, :b]) == list(sm.cold[u]), u
    nxt, e_ref, c_ref = oracle.iterate(X, s, K, C, 9, sampling)
    assert (e, c) == (e_ref, c_ref)
    g = ctx.export()
    assert np.array_equal(g.ids.cpu().numpy(), nxt.ids)
    assert np.array_equal(g.dists.cpu().numpy().astype(np.float64), nxt.dists)
    assert np.array_equal(g.flags.cpu().numpy(), nxt.flags)
    ctx.close()


@pytest.mark.parametrize("N,d,K,rho,hi,seed,path", [
    (600, 8, 10, 0.8, 12, 3, "valu"),
    (1000, 3, 15, 0.5, 40, 5, "valu"),
    (700, 64, 10, 1.0, 9, 1, "mfma"),
    (600, 100, 20, 0.5, 15, 2, "bf16x3"),
    (900, 130, 16, 1.0, 5, 3, "bf16x3"),
])
def test_turbo_build_integer_points_bitwise(knng, N, d, K, rho, hi, seed, path):
    X = synth.integer_points(N, d, hi, seed)
    ref = oracle.build_graph(X, K, rho, 0.001, 15, seed, sampling="turbo")
    ids, dists, st = knng.build(dev(X), K, rho, 0.001, 15, seed, path=path, sampling="turbo")
    assert st["iters"] == ref.iters
    assert st["evals"] == ref.evals.tolist()
    assert st["changes"] == ref.changes.tolist()
    assert np.array_equal(ids.cpu().numpy(), ref.ids)
    assert np.array_equal(dists.cpu().numpy().astype(np.float64), ref.dists)


def test_turbo_batch_equals_single_builds(knng):
    rng = np.random.default_rng(4)
    data = []
    for i in range(12):
        n = int(rng.integers(150, 1200))
        d = (16, 64)[i % 2]
        s = int(rng.integers(0, 2**31 - 1))
        data.append((synth.gaussian_mixture(n, d, 8, s), s))
    Xs = [dev(X) for X, _ in data]
    b = knng.Batch(Xs, [s for _, s in data], 15, 1.0, 0.001, 30, tuning="16:valu,64:bf16x3",
                   sampling="turbo")
    b.execute()
    b.synchronize()
    for i, (X, s) in enumerate(data):
        ids, dists, _ = knng.build(Xs[i], 15, 1.0, 0.001, 30, s, path="valu" if X.shape[1] == 16 else "bf16x3",
                                   sampling="turbo")
        assert torch.equal(b.ids[i], ids), i
        assert torch.equal(b.dists[i], dists), i


@pytest.mark.parametrize("K,rho,path", [(40, 1.0, "valu"), (64, 0.5, "mfma"), (48, 1.0, "valu")])
def test_turbo_large_caps_bitwise(knng, K, rho, path):
    """Caps above 30 (the rank-based large-pool select) on integer data."""
    X = synth.integer_points(1200, 16 if path == "valu" else 64, 9, 6)
    ref = oracle.build_graph(X, K, rho, 0.001, 12, 6, sampling="turbo")
    ids, dists, st = knng.build(dev(X), K, rho, 0.001, 12, 6, path=path, sampling="turbo")
    assert st["iters"] == ref.iters
    assert st["evals"] == ref.evals.tolist()
    assert st["changes"] == ref.changes.tolist()
    assert np.array_equal(ids.cpu().numpy(), ref.ids)
    assert np.array_equal(dists.cpu().numpy().astype(np.float64), ref.dists)


def test_image60k_turbo_bitwise(knng):
    """The benchmark workload (60000 x 784 pixel integers, K = 20, rho = 1)
    with turbosampling: the whole graph, e_t and c_t equal the oracle's."""
    X, p = synth.workload("image60k_d784")
    ref = oracle.build_graph(X, p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"], sampling="turbo")
    ids, dists, st = knng.build(dev(X), p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"],
                                sampling="turbo")
    assert st["converged"]
    assert st["iters"] == ref.iters
    assert st["evals"] == ref.evals.tolist()
    assert st["changes"] == ref.changes.tolist()
    assert np.array_equal(ids.cpu().numpy(), ref.ids)
    assert np.array_equal(dists.cpu().numpy().astype(np.float64), ref.dists)
