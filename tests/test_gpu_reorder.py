"""The device's graph-ordered permutation against the paper's greedy
clustering heuristic (Sec. 3.2, Algorithm 1; the oracle's host reference),
both built from the same G_1: window purity (Sec. 4, Fig. 4), label runs and
the span of list edges in memory. One JSON line per case is printed (run
with -s to see it).
"""
import json

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


def _purity(labels, w=2000, stride=1024):
    lab = labels - labels.min()
    n = int(lab.max()) + 1
    return np.array([np.bincount(lab[s:s + w], minlength=n).max() / w for s in range(0, len(lab) - w + 1, stride)])


def _locality(order, labels, ids):
    """order: node at each memory position."""
    N = len(order)
    pos = np.empty(N, np.int64)
    pos[order] = np.arange(N)
    seq = labels[order]
    span = np.abs(pos[:, None] - pos[ids])
    pur = _purity(seq)
    q = max(1, len(pur) // 4)
    return {"label_changes": int((seq[1:] != seq[:-1]).sum()),
            "purity_first_half": round(float(pur[:len(pur) // 2].mean()), 3),
            "purity_last_quarter": round(float(pur[-q:].mean()), 3),
            "edges_within_256": round(float((span < 256).mean()), 4),
            "median_edge_span": int(np.median(span))}


CASES = {
    # Fig. 4 setting: n = 16384, d = 8, 8 clusters; Fig. 5 setting: 16 clusters
    "clustered16k_8c": (lambda: synth.clustered_labels(16384, 8, 8, 3), 20, True),
    "clustered16k_16c": (lambda: synth.clustered_labels(16384, 8, 16, 4), 20, True),
    # low-d blobs with uniform background (the 4M-point workload's shape, smaller)
    "blobs200k_d3": (lambda: synth.lowd_blobs(200_000, 2, n_blobs=50, return_labels=True), 15, False),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_device_permutation_vs_greedy_heuristic(knng, case):
    gen, K, clustered = CASES[case]
    X, lab = gen()
    N = X.shape[0]
    ctx = knng.Context(torch.from_numpy(np.ascontiguousarray(X, np.float32)).to("cuda:0"), K, rho=1.0, seed=1,
                       reorder=True)
    ctx.init()
    ctx.iterate()                       # the permutation is applied after iteration 1
    order_dev = ctx.order().cpu().numpy()
    g1 = ctx.export().ids.cpu().numpy()
    ctx.close()
    assert np.array_equal(np.sort(order_dev), np.arange(N))
    _, order_alg1 = oracle.greedy_order(g1)
    res = {"case": case, "N": N, "K": K,
           "input_order": _locality(np.arange(N), lab, g1),
           "greedy_alg1": _locality(order_alg1, lab, g1),
           "device": _locality(order_dev, lab, g1)}
    print(json.dumps(res), flush=True)
    if clustered:
        assert res["device"]["label_changes"] <= res["greedy_alg1"]["label_changes"]
        assert res["device"]["purity_first_half"] >= res["greedy_alg1"]["purity_first_half"]
    assert res["device"]["edges_within_256"] > 5 * res["input_order"]["edges_within_256"]
    assert res["greedy_alg1"]["edges_within_256"] > 5 * res["input_order"]["edges_within_256"]
