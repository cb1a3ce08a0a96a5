"""The allocation-free entry point (knng_build_noalloc) against knng_build.

Its workspace is a static device array of the library; two calls in a row
(the second on a smaller input, so the array holds the first call's state
beyond what the second writes) must each give the graph, e_t and c_t of
knng_build on the same input bit for bit; a build that does not fit is
refused before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def knng():
    import paper_2112_06630_amd as k
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return k


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X, np.float32)).to("cuda:0")


CASES = [
    # (X, K, rho, seed, path, reorder): a matrix-path build with the permutation
    # after iteration 2 first, then a smaller direct-form build
    (lambda: synth.gaussian_mixture(3000, 64, 12, 31), 15, 1.0, 31, "auto", 2),
    (lambda: synth.gaussian_mixture(700, 16, 6, 32), 10, 0.5, 32, "auto", 0),
]


def _check_case(knng, X, K, rho, seed, path, reorder):
    Xd = _dev(X)
    N = X.shape[0]
    ids = torch.full((N, K), -7, dtype=torch.int32, device="cuda:0")
    dists = torch.full((N, K), -7.0, dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    st = knng.build_noalloc(Xd, K, ids, dists, rho, 0.001, 30, seed, reorder=reorder, path=path)
    torch.cuda.synchronize()
    ri, rd, rs = knng.build(Xd, K, rho, 0.001, 30, seed, reorder=reorder, path=path)
    assert torch.equal(ids, ri) and torch.equal(dists, rd)
    assert st["iters"] == rs["iters"] and st["converged"] == rs["converged"]
    assert st["evals"] == rs["evals"] and st["changes"] == rs["changes"]
    assert st["path"] == rs["path"] and st["total_ms"] == 0.0


def test_noalloc_two_calls_match_build(knng):
    for gen, K, rho, seed, path, reorder in CASES:
        _check_case(knng, gen(), K, rho, seed, path, reorder)


def test_noalloc_refuses_what_does_not_fit(knng):
    X = _dev(synth.gaussian_mixture(50000, 16, 10, 3))
    ids = torch.empty((50000, 20), dtype=torch.int32, device="cuda:0")
    dists = torch.empty((50000, 20), dtype=torch.float32, device="cuda:0")
    with pytest.raises(knng.KnngError) as e:
        knng.build_noalloc(X, 20, ids, dists)
    assert e.value.status == 2 and "static scratch" in str(e.value)
    # the refusal leaves the entry point usable
    _check_case(knng, synth.gaussian_mixture(500, 8, 4, 5), 8, 1.0, 5, "valu", 0)
