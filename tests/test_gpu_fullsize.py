"""Parity at the benchmark sizes, in the launch configuration bench.py times.

image60k_d784 (60000 x 784 pixel integers, K=20, rho=1): every distance is an
exact integer below 2^24 in FP32 and in the split-BF16 form, so the whole
GPU graph, e_t and c_t must equal the FP64 oracle's full build bit for bit (about 15 s of oracle on 8
host threads).

audio54k_d192 (an audio-shaped stand-in, 54387 x 192 continuous features,
K=20, rho=1): one iteration from the oracle's G_0 against its G_1 within the
FP32 Gram-form bound, and the whole build checked on sampled rows against
brute force and against the oracle's own build.

blobs4m_d3 and aniso200k_d960 are too large for a full oracle build in a test;
their sampled rows are checked one by one against brute force from the
oracle: stored distances within the FP32 bound, rows sorted, distinct, no
self, and the recall of the sample.
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
    res = check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), s1.ids, s1.dists, dpad=192, gram=True)
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
