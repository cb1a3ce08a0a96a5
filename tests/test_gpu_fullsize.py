"""Parity at the benchmark sizes, in the launch configuration bench.py times.

image60k_d784 (60000 x 784 pixel integers, K=20, rho=1): every distance is an
exact integer below 2^24 in FP32 and in the split-BF16 form, so the whole
GPU graph, e_t and c_t must equal the FP64 oracle's full build bit for bit (about 15 s of oracle on 8
host threads).

blobs4m_d3 (4M x 3) and aniso200k_d960 (200000 x 960, plain and BF16-screened):
one iteration from the oracle's G_0 against its G_1 at full size (sampled
sets exact, e_1 exact, ids equal except at ties within 1e-5 relative); the
whole builds are checked on sampled rows against brute force from the oracle
(stored distances within the FP32 bound, rows sorted, distinct, no self, the
recall of the sample).

audio54k_d192 (an audio-shaped stand-in, 54387 x 192 continuous features,
K=20, rho=1): one iteration from the oracle's G_0 against its G_1, and the
whole build checked on sampled rows against brute force and against the
oracle's own build.

batch512: the full batch against one single build per dataset, bit for bit.
The split form at d = 3144 (the top of the paper's dimension sweep): step
parity against the oracle at N = 2000.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import check_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def knng():
    import paper_2112_06630_amd as k
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return k


@pytest.fixture(scope="module")
def image60k():
    X, p = synth.workload("image60k_d784")
    ref = oracle.build_graph(X, p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"])
    return X, p, ref


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X, np.float32)).to("cuda:0")


@pytest.mark.parametrize("path,reorder,want", [
    ("auto", False, 4),    # split-BF16 Gram tiles: what the benchmark runs
    ("auto", True, 4),     # with the graph-ordered permutation
    ("mfma", False, 2),    # FP32 Gram tiles
])
def test_image60k_bitwise(knng, image60k, path, reorder, want):
    X, p, ref = image60k
    ids, dists, st = knng.build(_dev(X), p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"],
                                path=path, reorder=reorder)
    assert st["path"] == want
    assert st["accurate"] == 0   # 0..255 integers, squared norms below 2^23: FP32 sums exact
    assert st["u8"] == (1 if want == 4 else 0)   # the split form reads them as byte rows
    assert st["converged"]
    assert st["iters"] == ref.iters
    assert st["evals"] == ref.evals.tolist()
    assert st["changes"] == ref.changes.tolist()
    assert np.array_equal(ids.cpu().numpy(), ref.ids)
    assert np.array_equal(dists.cpu().numpy().astype(np.float64), ref.dists)


def _check_sampled(X, ids, dists, rows, K, dpad, gram, min_recall):
    gi = ids[rows]
    gd = dists[rows].astype(np.float64)
    assert (gi >= 0).all() and (gi < X.shape[0]).all()
    assert not (gi == rows[:, None]).any(), "self in a row"
    assert all(len(set(r.tolist())) == K for r in gi), "duplicate ids in a row"
    # stored distances vs FP64 recomputation, within the bound of the formula used
    D64 = np.array([[np.sum((X[r].astype(np.float64) - X[q].astype(np.float64)) ** 2) for q in gi[i]]
                    for i, r in enumerate(rows)])
    if gram:
        n = (X.astype(np.float64) ** 2).sum(1)
        bound = (dpad / 4 + 8) * 4 * 2.0 ** -24 * (n[rows][:, None] + n[gi]) + 1e-30
    else:
        bound = (dpad / 4 + 5) * 2 * 2.0 ** -24 * D64 + 1e-30
    assert (np.abs(gd - D64) <= bound).all()
    # sorted by (distance, id)
    assert ((gd[:, 1:] > gd[:, :-1]) | ((gd[:, 1:] == gd[:, :-1]) & (gi[:, 1:] > gi[:, :-1]))).all()
    ei, ed = oracle.bruteforce_rows(X, K, rows)
    hits = 0
    for i in range(len(rows)):
        tau = ed[i, -1]
        hits += int(np.sum(D64[i] <= tau * (1 + 1e-5)))
    rec = hits / (len(rows) * K)
    assert rec >= min_recall, rec
    return rec


def test_blobs4m_sampled_rows(knng):
    X, p = synth.workload("blobs4m_d3")
    ids, dists, st = knng.build(_dev(X), p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"])
    assert st["path"] == 1 and st["converged"]
    rows = np.random.default_rng(0).choice(X.shape[0], 256, replace=False)
    _check_sampled(X, ids.cpu().numpy(), dists.cpu().numpy(), rows, p["K"], 4, False, 0.99)


def test_aniso200k_sampled_rows(knng):
    X, p = synth.workload("aniso200k_d960")
    ids, dists, st = knng.build(_dev(X), p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"])
    assert st["path"] == knng.PATH_MFMA_BF16X3
    rows = np.random.default_rng(1).choice(X.shape[0], 128, replace=False)
    _check_sampled(X, ids.cpu().numpy(), dists.cpu().numpy(), rows, p["K"], 960, True, 0.5)


def test_audio54k_step_and_build(knng):
    X = synth.audio_like(54387, 192, 7)
    K, rho, delta, T, seed = 20, 1.0, 0.001, 30, 7
    C = oracle.cap(K, rho)
    s0 = oracle.init(X, K, seed)
    s1, e1, _ = oracle.iterate(X, s0, K, C, seed)
    ctx = knng.Context(_dev(X), K, rho, delta, T, seed)
    ctx.load(torch.from_numpy(s0.ids), torch.from_numpy(s0.flags), 0)
    eg, _ = ctx.iterate()
    assert eg == e1
    g = ctx.export()
    res = check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), s1.ids, s1.dists, dpad=192, gram=True,
                     accurate=True)
    assert res["exact_rows"] >= X.shape[0] - 60, res
    ctx.close()
    ids, dists, st = knng.build(_dev(X), K, rho, delta, T, seed)
    assert st["path"] == knng.PATH_MFMA_BF16X3 and st["converged"]
    rows = np.random.default_rng(2).choice(X.shape[0], 400, replace=False)
    rec = _check_sampled(X, ids.cpu().numpy(), dists.cpu().numpy(), rows, K, 192, True, 0.9)
    ref = oracle.build_graph(X, K, rho, delta, T, seed)
    _, ed = oracle.bruteforce_rows(X, K, rows)
    ref_rec = float(np.mean(ref.dists[rows] <= ed[:, -1:] * (1 + 1e-5)))
    assert rec >= ref_rec - 0.01, (rec, ref_rec)


def _samples_equal(ctx, sm_arrays):
    """GPU sampled sets of the last iteration against the oracle's, exactly."""
    cnew, nnew, cold, nold, _ = sm_arrays
    nw, od, cnt = (a.cpu().numpy() for a in ctx.samples())
    assert np.array_equal(cnt[:, 0], nnew) and np.array_equal(cnt[:, 1], nold)
    C = cnew.shape[1]
    col = np.arange(C)[None, :]
    assert np.array_equal(np.where(col < nnew[:, None], nw, -1), np.where(col < nnew[:, None], cnew, -1))
    assert np.array_equal(np.where(col < nold[:, None], od, -1), np.where(col < nold[:, None], cold, -1))


def test_blobs4m_oracle_step(knng):
    """4M x 3 low-d blobs at full size, in the launch configuration the bench
    times (AUTO: direct form): one GPU iteration from the oracle's G_0 against
    its G_1 -- sampled sets integer-exact (the counting-sort reverse lists
    over super-buckets of 2^9 positions, some 7800 of them), e_1 exact, ids
    equal except at ties within 1e-5 relative."""
    X, p = synth.workload("blobs4m_d3")
    K, rho, seed = p["K"], p["rho"], p["seed"]
    C = oracle.cap(K, rho)
    s0 = oracle.init(X, K, seed)
    sm = oracle.sample_arrays(s0, K, C, seed, 1)
    s1, e1, _ = oracle.iterate(X, s0, K, C, seed)
    ctx = knng.Context(_dev(X), K, rho, p["delta"], p["max_iters"], seed)
    assert ctx.stats()["path"] == knng.PATH_VALU
    ctx.load(torch.from_numpy(s0.ids), torch.from_numpy(s0.flags), 0)
    eg, _ = ctx.iterate()
    assert eg == e1
    _samples_equal(ctx, sm)
    g = ctx.export()
    res = check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), s1.ids, s1.dists, dpad=4)
    assert res["exact_rows"] >= X.shape[0] - 100, res
    ctx.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_aniso200k_oracle_step(knng, precision):
    """200000 x 960 anisotropic clusters at full size, plain (split form,
    three planes, FP64 accumulation) and the BF16-screened form: one GPU
    iteration from the oracle's G_0 against its G_1 -- sampled sets exact, e_1
    exact, ids equal except at ties within 1e-5 relative, stored distances
    within the bound of the form used."""
    X, p = synth.workload("aniso200k_d960")
    K, rho, seed = p["K"], p["rho"], p["seed"]
    C = oracle.cap(K, rho)
    s0 = oracle.init(X, K, seed)
    sm = oracle.sample_arrays(s0, K, C, seed, 1)
    s1, e1, _ = oracle.iterate(X, s0, K, C, seed)
    ctx = knng.Context(_dev(X), K, rho, p["delta"], p["max_iters"], seed, precision=precision)
    st = ctx.stats()
    if precision == "fp32":
        assert st["path"] == knng.PATH_MFMA_BF16X3 and st["planes"] == 3 and st["accurate"] == 1
    ctx.load(torch.from_numpy(s0.ids), torch.from_numpy(s0.flags), 0)
    eg, _ = ctx.iterate()
    assert eg == e1
    _samples_equal(ctx, sm)
    g = ctx.export()
    gram = precision == "fp32"
    res = check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), s1.ids, s1.dists, dpad=960, gram=gram,
                     accurate=gram)
    assert res["exact_rows"] >= X.shape[0] - 100, res
    ctx.close()


def test_split_form_d3144_step_parity(knng):
    """The top of the paper's dimension sweep (Sec. 4.5: d up to 3144) on its
    single Gaussian, N = 2000: one GPU iteration of the split form (three
    planes, FP64 accumulation) from every oracle state G_t against G_{t+1}."""
    X = synth.single_gaussian(2000, 3144, 5)
    K, rho, seed = 10, 1.0, 5
    r = oracle.build_graph(X, K, rho, 0.0, 4, seed, keep_states=True)
    for s, nxt, e in zip(r.states[:-1], r.states[1:], r.evals):
        ctx = knng.Context(_dev(X), K, rho=rho, seed=seed, path="bf16x3")
        assert ctx.stats()["planes"] == 3 and ctx.stats()["dpad"] == 3168
        ctx.load(torch.from_numpy(s.ids), torch.from_numpy(s.flags), s.t)
        eg, _ = ctx.iterate()
        assert eg == e
        g = ctx.export()
        res = check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), nxt.ids, nxt.dists, dpad=3168, gram=True,
                         accurate=True)
        assert res["exact_rows"] >= X.shape[0] - 10, (s.t, res)
        ctx.close()


def test_batch512_equals_sequential_builds(knng):
    """The full 512-dataset batch (N log-uniform in [500, 20000], d in
    {16, 64, 128}), in the configuration the bench times (autotuned table,
    captured graph): every dataset's graph, e_t and c_t equal a single build
    of it on the same join path, bit for bit."""
    data = synth.batched_datasets(512, 4)
    Xs = [_dev(X) for X, _ in data]
    seeds = [s for _, s in data]
    b = knng.Batch(Xs, seeds, 15, 1.0, 0.001, 30)
    entries = {d: r.partition("@")[0] for d, r in (e.split(":") for e in b.tuning.split(","))}
    b.capture()
    b.launch()
    b.synchronize()
    st = b.stats()
    for i, (X, s) in enumerate(zip(Xs, seeds)):
        ids, dists, ss = knng.build(X, 15, 1.0, 0.001, 30, s, path=entries[str(X.shape[1])])
        assert torch.equal(b.ids[i], ids) and torch.equal(b.dists[i], dists), i
        assert st["evals"][i] == ss["evals"] and st["changes"][i] == ss["changes"], i
    b.close()
