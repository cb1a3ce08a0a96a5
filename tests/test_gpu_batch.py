"""Batched form: many datasets in one (graph) launch must equal one build per dataset."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def knng():
    import paper_2112_06630_amd as k
    assert torch.cuda.is_available()
    return k


def small_batch(count, seed, dims=(16, 64, 128), n_lo=100, n_hi=1500):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        d = int(dims[int(rng.integers(0, len(dims)))])
        s = int(rng.integers(0, 2**31 - 1))
        out.append((synth.gaussian_mixture(n, d, int(rng.integers(5, 21)), s), s))
    return out


def dev(X):
    return torch.from_numpy(np.ascontiguousarray(X, np.float32)).to("cuda:0")


TABLE = "16:valu,64:mfma,128:valu"


def path_for(d):
    return {16: "valu", 64: "mfma", 128: "valu"}[d]


@pytest.mark.parametrize("table", [TABLE, "16:bf16x3,64:bf16x3,128:bf16x3", "16:mfma,64:valu,128:mfma"])
def test_batch_equals_single_builds(knng, table):
    data = small_batch(24, 11)
    Xs = [dev(X) for X, _ in data]
    seeds = [s for _, s in data]
    b = knng.Batch(Xs, seeds, 15, 1.0, 0.001, 30, tuning=table)
    assert b.tuning == table
    path_for = lambda d: dict(e.split(":") for e in table.split(","))[str(d)]
    b.execute()
    b.synchronize()
    st = b.stats()
    for i, (X, s) in enumerate(data):
        ids, dists, ss = knng.build(Xs[i], 15, 1.0, 0.001, 30, s, path=path_for(X.shape[1]))
        assert torch.equal(b.ids[i], ids) and torch.equal(b.dists[i], dists), i
        assert st["iters"][i] == ss["iters"] and st["evals"][i] == ss["evals"] and st["changes"][i] == ss["changes"]
        assert bool(st["converged"][i]) == ss["converged"]
    b.close()


@pytest.mark.parametrize("tuning", ["16:valu,64:mfma,128:mfma", "16:valu,64:bf16x3,128:bf16x3"])
def test_batch_integer_data_matches_oracle(knng, tuning):
    rng = np.random.default_rng(3)
    data = [(synth.integer_points(int(n), int(d), 7, int(s)), int(s))
            for n, d, s in zip(rng.integers(60, 700, 6), [16, 16, 64, 64, 128, 128], rng.integers(0, 1000, 6))]
    Xs = [dev(X) for X, _ in data]
    b = knng.Batch(Xs, [s for _, s in data], 10, 0.7, 0.001, 20, tuning=tuning)
    b.execute()
    b.synchronize()
    st = b.stats()
    for i, (X, s) in enumerate(data):
        ref = oracle.build_graph(X, 10, 0.7, 0.001, 20, s)
        assert np.array_equal(b.ids[i].cpu().numpy(), ref.ids)
        assert np.array_equal(b.dists[i].cpu().numpy().astype(np.float64), ref.dists)
        assert st["changes"][i] == ref.changes.tolist()
    b.close()


def test_batch_bf16_exact_noninteger_matches_single(knng):
    """Values exact in BF16 but not integers (8-bit mantissas over eleven
    binades), so FP32 sums round: a single build reads the one BF16 plane
    that holds them, the batch the FP32 rows; both sum every dot product in
    the same dimension order, so the graphs agree bit for bit."""
    rng = np.random.default_rng(21)
    data = []
    for n, d, s in zip([400, 900, 650, 300], [64, 64, 128, 128], [5, 6, 7, 8]):
        m = rng.integers(128, 256, (n, d)).astype(np.float64)
        e = rng.integers(-10, 1, (n, d)).astype(np.float64)
        X = (m * 2.0 ** e * rng.choice([-1.0, 1.0], (n, d))).astype(np.float32)
        X[: n // 2, : d // 4] *= np.float32(8.0)   # two coarse groups (a power of two keeps BF16 exactness)
        data.append((X, s))
    Xs = [dev(X) for X, _ in data]
    b = knng.Batch(Xs, [s for _, s in data], 12, 1.0, 0.001, 20, tuning="64:bf16x3,128:bf16x3")
    b.execute()
    b.synchronize()
    st = b.stats()
    for i, (X, s) in enumerate(data):
        ids, dists, ss = knng.build(Xs[i], 12, 1.0, 0.001, 20, s, path="bf16x3")
        assert ss["planes"] == 1
        assert torch.equal(b.ids[i], ids) and torch.equal(b.dists[i], dists), i
        assert st["evals"][i] == ss["evals"] and st["changes"][i] == ss["changes"]
    b.close()


def test_batch_graph_replays(knng):
    """Captured graph, replayed three times with eager work in between: every
    replay must equal the eager execution."""
    data = small_batch(10, 5)
    Xs = [dev(X) for X, _ in data]
    b = knng.Batch(Xs, [s for _, s in data], 15, 1.0, 0.001, 30, tuning=TABLE)
    b.execute()
    b.synchronize()
    ref_ids = [t.clone() for t in b.ids]
    ref_d = [t.clone() for t in b.dists]
    b.capture()
    for rep in range(3):
        for t in b.ids:
            t.fill_(-1)
        torch.cuda.synchronize()
        b.launch()
        b.synchronize()
        for i in range(len(Xs)):
            assert torch.equal(b.ids[i], ref_ids[i]) and torch.equal(b.dists[i], ref_d[i]), (rep, i)
        _ = (Xs[0] * 2).sum().item()   # unrelated eager work between replays
    b.close()


def test_batch_autotune_table(knng):
    data = small_batch(9, 7)
    Xs = [dev(X) for X, _ in data]
    b = knng.Batch(Xs, [s for _, s in data], 15, 1.0, 0.001, 30)
    table = b.tuning
    # "d:path" or "d:path@cap" (workgroup cap of the select and join passes)
    entries = {d: rest.partition("@")[0] for d, rest in (e.split(":") for e in table.split(","))}
    assert set(entries) == {str(X.shape[1]) for X, _ in data}
    assert set(entries.values()) <= {"valu", "mfma", "bf16x3"}
    b.execute()
    b.synchronize()
    for i, (X, s) in enumerate(data):
        ids, dists, _ = knng.build(Xs[i], 15, 1.0, 0.001, 30, s, path=entries[str(X.shape[1])])
        assert torch.equal(b.ids[i], ids), i
    b.close()


def test_batch_rejects_bad_input(knng):
    X = synth.integer_points(100, 16, 5, 1)
    X[3, 3] = np.nan
    with pytest.raises(knng.KnngError):
        knng.Batch([dev(X)], [1], 10, tuning="16:valu")
    with pytest.raises(knng.KnngError):
        knng.Batch([dev(synth.integer_points(8, 16, 5, 1))], [1], 10, tuning="16:valu")  # K > N-1


def test_batch_of_tiny_datasets(knng):
    """Groups of a few dozen points (fewer join workgroups than XCDs) still
    match their single builds."""
    data = [(synth.integer_points(n, d, 7, 60 + n), 60 + n) for n, d in [(3, 16), (9, 16), (12, 64), (5, 64)]]
    Xs = [dev(X) for X, _ in data]
    seeds = [s for _, s in data]
    b = knng.Batch(Xs, seeds, 2, 1.0, 0.001, 10, tuning="16:valu,64:bf16x3")
    b.execute()
    b.synchronize()
    for i, (X, s) in enumerate(data):
        ids, dists, _ = knng.build(Xs[i], 2, 1.0, 0.001, 10, s, path="valu" if X.shape[1] == 16 else "bf16x3")
        assert torch.equal(b.ids[i], ids) and torch.equal(b.dists[i], dists), i
        ref = oracle.build_graph(X, 2, 1.0, 0.001, 10, s)
        assert np.array_equal(ids.cpu().numpy(), ref.ids), i
    b.close()


def test_batch_launch_shape_does_not_change_results(knng):
    """The workgroup cap of the select and join passes ("@n" in the tuning
    table) changes only how owners are spread over workgroups."""
    data = small_batch(10, 21)
    Xs = [dev(X) for X, _ in data]
    seeds = [s for _, s in data]
    out = []
    for table in ["16:valu,64:bf16x3,128:mfma", "16:valu@64,64:bf16x3@7,128:mfma@300"]:
        b = knng.Batch(Xs, seeds, 15, 1.0, 0.001, 30, tuning=table)
        assert b.tuning == table
        b.execute()
        b.synchronize()
        out.append(([t.clone() for t in b.ids], [t.clone() for t in b.dists], b.stats()))
        b.close()
    for i in range(len(data)):
        assert torch.equal(out[0][0][i], out[1][0][i]) and torch.equal(out[0][1][i], out[1][1][i]), i
    assert out[0][2]["evals"] == out[1][2]["evals"]


def test_autotuner_table_is_valid(knng):
    data = small_batch(6, 23)
    b = knng.Batch([dev(X) for X, _ in data], [s for _, s in data], 15, 1.0, 0.001, 30)
    for item in b.tuning.split(","):
        d, rest = item.split(":")
        path, _, cap = rest.partition("@")
        assert path in ("valu", "mfma", "bf16x3") and (cap == "" or int(cap) > 0)
    b.close()
