"""GPU path vs the FP64 oracle, through the C ABI (ctypes binding).

Integer-coordinate inputs make every FP32 sum exact, so there the GPU graph
must equal the oracle's bit for bit (ids, distances, e_t, c_t per
iteration). Continuous inputs follow the tie-aware rule in tests/parity.py.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import check_rows, fp32_bound

pytestmark = pytest.mark.gpu

# The exact integer form (int8 MFMA) was withdrawn from the library: its first
# GPU run ended in a device fault whose cause has not been found, so its
# tests stay skipped until one is.
I8_OFF = pytest.mark.skip(reason="exact integer form withdrawn (unresolved device fault)")


@pytest.fixture(scope="module")
def knng():
    import paper_2112_06630_amd as k
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return k


def dev(X):
    return torch.from_numpy(np.ascontiguousarray(X, np.float32)).to("cuda:0")


def exact_build(knng, X, K, rho, delta, T, seed, path="auto", reorder=False):
    ref = oracle.build_graph(X, K, rho, delta, T, seed)
    ids, dists, st = knng.build(dev(X), K, rho, delta, T, seed, reorder=reorder, path=path)
    ids = ids.cpu().numpy()
    dists = dists.cpu().numpy().astype(np.float64)
    assert st["iters"] == ref.iters
    assert st["evals"] == ref.evals.tolist()
    assert st["changes"] == ref.changes.tolist()
    assert np.array_equal(ids, ref.ids)
    assert np.array_equal(dists, ref.dists)
    return st


@pytest.mark.parametrize("N,d,K,rho,hi,seed", [
    (600, 8, 10, 0.8, 12, 3),
    (1000, 3, 15, 0.5, 40, 5),
    (777, 16, 7, 1.0, 6, 11),
    (500, 1, 5, 1.0, 300, 2),
])
def test_build_integer_points_bitwise_valu(knng, N, d, K, rho, hi, seed):
    st = exact_build(knng, synth.integer_points(N, d, hi, seed), K, rho, 0.001, 15, seed, path="valu")
    assert st["path"] == knng.PATH_VALU


@pytest.mark.parametrize("N,d,K,rho,hi,seed", [
    (700, 64, 10, 1.0, 9, 1),
    (600, 100, 20, 0.5, 15, 2),
    (900, 130, 16, 1.0, 5, 3),
    (400, 33, 12, 0.9, 20, 4),
])
@pytest.mark.parametrize("path", ["mfma", "bf16x3"])
def test_build_integer_points_bitwise_mfma(knng, N, d, K, rho, hi, seed, path):
    st = exact_build(knng, synth.integer_points(N, d, hi, seed), K, rho, 0.001, 15, seed, path=path)
    assert st["path"] == (knng.PATH_MFMA if path == "mfma" else knng.PATH_MFMA_BF16X3)


@pytest.mark.parametrize("path,want", [("auto", 4), ("mfma", 2)])
def test_image_like_subset_bitwise(knng, path, want):
    """784-d 0..255 integer data (image-shaped workload at N=3000): exact in
    FP32 and in the split-BF16 form (x1 = x, x2 = x3 = 0), which AUTO takes."""
    X = synth.image_like(3000, 1)
    st = exact_build(knng, X, 20, 1.0, 0.001, 30, 1, path=path)
    assert st["path"] == want
    assert st["planes"] == (1 if want == 4 else 0)   # pixels are exact in BF16: one plane
    assert st["u8"] == (1 if want == 4 else 0)       # ... read as bytes


@pytest.mark.parametrize("bits,planes", [(8, 1), (12, 2), (16, 2), (24, 3)])
def test_split_plane_count(knng, bits, planes):
    """Values with at most 8 significant bits need one BF16 plane, at most 16
    two, else three: the join reads only planes that are not all zero."""
    rng = np.random.default_rng(bits)
    X = rng.integers(0, 2 ** bits, (300, 64)).astype(np.float32)
    _, _, st = knng.build(dev(X), 8, max_iters=2, path="bf16x3")
    assert st["planes"] == planes


@pytest.mark.parametrize("shift,want_u8", [(0, 1), (-1, 0), (56, 0)])
def test_byte_rows_only_for_8bit_data(knng, shift, want_u8):
    """Integers in 0..255 with exact FP32 sums are read as byte rows (half the
    bytes of the BF16 plane, widened in registers); other exact integer data
    (a negative value; 256, still one BF16 plane) keeps the plane. Both reproduce the
    oracle bit for bit."""
    X = (synth.integer_points(700, 64, 200, 9) + np.float32(shift)).astype(np.float32)
    st = exact_build(knng, X, 10, 1.0, 0.001, 15, 9, path="bf16x3")
    assert st["planes"] == 1 and st["accurate"] == 0 and st["u8"] == want_u8


def test_split_two_planes_step_parity(knng):
    """12-bit integers (two planes; FP32 sums round above 2^24): one GPU
    iteration per oracle state, tie-aware parity with the Gram-form bound."""
    X = np.random.default_rng(13).integers(0, 4096, (2000, 80)).astype(np.float32)
    X[:1000] += 2048.0 * (np.arange(80) % 3 == 0)   # two coarse groups
    r = oracle.build_graph(X, 12, 1.0, 0.0, 5, 2, keep_states=True)
    for s, nxt, e in zip(r.states[:-1], r.states[1:], r.evals):
        ctx = knng.Context(dev(X), 12, rho=1.0, seed=2, path="bf16x3")
        assert ctx.stats()["planes"] == 2
        assert ctx.stats()["accurate"] == 1   # squared norms above 2^23: FP32 sums round
        ctx.load(torch.from_numpy(s.ids), torch.from_numpy(s.flags), s.t)
        eg, _ = ctx.iterate()
        assert eg == e
        g = ctx.export()
        res = check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), nxt.ids, nxt.dists, dpad=96, gram=True,
                         accurate=True)
        assert res["exact_rows"] >= 2000 - 10
        ctx.close()


# ----------------------------------------------------------------- split-BF16 Gram form

def _split_case(gen):
    if gen == "aniso":
        return synth.anisotropic_clusters(3000, 960, 3, 20), 20, 0.5, 3
    if gen == "gauss":
        return synth.gaussian_mixture(4000, 128, 12, 9), 16, 1.0, 9
    return synth.gaussian_mixture(3000, 96, 10, 10), 32, 1.0, 10


@pytest.mark.parametrize("gen,path", [("aniso", "bf16x3"), ("gauss", "bf16x3"), ("gauss_wide", "bf16x3"),
                                      ("gauss", "mfma"), ("gauss_wide", "mfma")])
def test_split_form_step_parity(knng, gen, path):
    """Continuous data, one GPU iteration from each oracle state G_t against
    the oracle's G_{t+1}: ids equal except at ties within 1e-5 relative, rows
    in FP64 order up to such ties, distances within the bound of the FP64-
    accumulated Gram form, e_t exact. The Gaussian mixtures sit far from the
    origin (||x||^2 about 17 times the neighbour distances), where an FP32
    Gram form errs by more than 1e-5 of the distance. (Over a whole build a
    near-tie decided differently from FP64 changes the later samples, so
    whole builds are compared by the bound and by recall below.) A pair
    proposed by several owners must carry one key, else the merge reports a
    duplicate id: this also checks that the distance is symmetric. gauss_wide
    has 2C = 64 columns (the four-column-tile kernels)."""
    X, K, rho, seed = _split_case(gen)
    dpad = (X.shape[1] + 31) // 32 * 32
    r = oracle.build_graph(X, K, rho, 0.0, 6, seed, keep_states=True)
    for s, nxt, e in zip(r.states[:-1], r.states[1:], r.evals):
        ctx = knng.Context(dev(X), K, rho=rho, seed=seed, path=path)
        assert ctx.stats()["accurate"] == 1
        ctx.load(torch.from_numpy(s.ids), torch.from_numpy(s.flags), s.t)
        eg, cg = ctx.iterate()
        assert eg == e
        g = ctx.export()
        res = check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), nxt.ids, nxt.dists, dpad=dpad, gram=True,
                         accurate=True)
        assert res["exact_rows"] >= X.shape[0] - 10, (s.t, res)
        ctx.close()


@pytest.mark.parametrize("gen", ["aniso", "gauss", "gauss_wide"])
def test_split_form_whole_build(knng, gen):
    """Whole build: rows valid and sorted, stored distances within the FP32
    Gram-form bound, recall as the oracle's (within 0.005)."""
    X, K, rho, seed = _split_case(gen)
    dpad = (X.shape[1] + 31) // 32 * 32
    ids, dists, st = knng.build(dev(X), K, rho, 0.001, 30, seed, path="bf16x3")
    assert st["path"] == knng.PATH_MFMA_BF16X3 and st["accurate"] == 1
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    D64, bound = fp32_bound(X, ids, dpad, True, accurate=True)
    assert (np.abs(dists.astype(np.float64) - D64) <= bound).all()
    assert all(len(set(r.tolist())) == K for r in ids)
    assert not (ids == np.arange(X.shape[0])[:, None]).any()
    assert ((dists[:, 1:] > dists[:, :-1]) | ((dists[:, 1:] == dists[:, :-1]) & (ids[:, 1:] > ids[:, :-1]))).all()
    ref = oracle.build_graph(X, K, rho, 0.001, 30, seed)
    ei, ed = oracle.bruteforce(X, K)
    assert oracle.recall(X, ids, ed) >= oracle.recall(X, ref.ids, ed) - 0.005


def test_split_form_wide_exponent_range(knng):
    """Values spread over many binades (log-uniform magnitudes, random signs):
    the split must stay exact term by term; step parity as above."""
    rng = np.random.default_rng(12)
    X = (rng.choice([-1.0, 1.0], (2500, 96)) * 10.0 ** rng.uniform(-6, 3, (2500, 96))).astype(np.float32)
    X[:, :8] += rng.integers(0, 5, (2500, 1)).astype(np.float32) * 1000.0   # clustered on a few axes
    r = oracle.build_graph(X, 12, 1.0, 0.0, 4, 4, keep_states=True)
    for s, nxt in zip(r.states[:-1], r.states[1:]):
        ctx = knng.Context(dev(X), 12, rho=1.0, seed=4, path="bf16x3")
        ctx.load(torch.from_numpy(s.ids), torch.from_numpy(s.flags), s.t)
        ctx.iterate()
        g = ctx.export()
        res = check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), nxt.ids, nxt.dists, dpad=96, gram=True,
                         accurate=True)
        assert res["exact_rows"] >= 2500 - 10
        ctx.close()


# ----------------------------------------------------------------- exact integer form (int8 MFMA)

@I8_OFF
@pytest.mark.parametrize("N,d,K,rho,lo,hi,seed", [
    (700, 64, 10, 1.0, 0, 255, 1),         # full 8-bit span
    (600, 100, 20, 0.5, -1000, -745, 2),   # negative, shifted span 255
    (900, 130, 16, 1.0, 3, 9, 3),          # narrow span, d not a multiple of 64
    (400, 33, 12, 0.9, 100, 300, 4),       # d < 64 on request
    (520, 257, 32, 1.0, -128, 127, 5),     # 2C = 64 columns, dpi = 320 (ragged k blocks)
])
def test_integer_form_bitwise(knng, N, d, K, rho, lo, hi, seed):
    """Every distance is exact, so the graph, e_t and c_t equal the oracle's bit for bit."""
    X = (synth.integer_points(N, d, hi - lo, seed) + np.float32(lo)).astype(np.float32)
    st = exact_build(knng, X, K, rho, 0.001, 15, seed, path="mfma_i8")
    assert st["path"] == knng.PATH_MFMA_I8


@I8_OFF
def test_integer_form_matches_fp32_paths(knng):
    """Where FP32 is exact too, the three join forms give identical graphs."""
    X = synth.integer_points(1200, 96, 40, 8)
    out = {p: knng.build(dev(X), 12, 1.0, 0.001, 15, 8, path=p) for p in ("valu", "mfma", "mfma_i8")}
    for p in ("mfma", "mfma_i8"):
        assert torch.equal(out[p][0], out["valu"][0]) and torch.equal(out[p][1], out["valu"][1])
        assert out[p][2]["changes"] == out["valu"][2]["changes"]


@I8_OFF
def test_integer_form_long_rows(knng):
    """d = 2000 at span 255: distances reach 1.3e8 > 2^24, stored as the
    correctly rounded exact value; parity with the FP64 oracle up to ties."""
    X = synth.integer_points(1000, 2000, 255, 6)
    ref = oracle.build_graph(X, 10, 1.0, 0.001, 12, 6)
    ids, dists, st = knng.build(dev(X), 10, 1.0, 0.001, 12, 6, path="auto")
    assert st["path"] == knng.PATH_MFMA_I8
    d64 = oracle.list_dists(X, ids.cpu().numpy())
    assert np.array_equal(dists.cpu().numpy(), d64.astype(np.float32))   # correctly rounded
    res = check_rows(X, ids.cpu().numpy(), dists.cpu().numpy(), ref.ids, ref.dists)
    assert res["exact_rows"] >= 1000 - 5


@I8_OFF
def test_integer_form_step_parity(knng):
    """Load each oracle state G_t (distances recomputed in the integer form),
    run one iteration, compare with the oracle's G_{t+1} bit for bit."""
    X = synth.image_like(1500, 3)
    K = 20
    r = oracle.build_graph(X, K, 1.0, 0.0, 6, 5, keep_states=True)
    for s, nxt, e, c in zip(r.states[:-1], r.states[1:], r.evals, r.changes):
        ctx = knng.Context(dev(X), K, rho=1.0, seed=5, path="mfma_i8")
        ctx.load(torch.from_numpy(s.ids), torch.from_numpy(s.flags), s.t)
        eg, cg = ctx.iterate()
        assert (eg, cg) == (e, c)
        g = ctx.export()
        assert np.array_equal(g.ids.cpu().numpy(), nxt.ids)
        assert np.array_equal(g.dists.cpu().numpy().astype(np.float64), nxt.dists)
        ctx.close()


def test_auto_path_choice(knng):
    """AUTO follows the crossover of the single-Gaussian sweeps: the direct
    form below d = 56, the split form from 56 (three planes on these values);
    integer pixel-like data (one plane) take the split form too."""
    for d, want in ((40, knng.PATH_VALU), (48, knng.PATH_VALU), (64, knng.PATH_MFMA_BF16X3),
                    (160, knng.PATH_MFMA_BF16X3), (224, knng.PATH_MFMA_BF16X3)):
        X = synth.single_gaussian(600, d, 3)
        _, _, st = knng.build(dev(X), 10, 1.0, 0.001, 3, 3, path="auto")
        assert st["path"] == want, (d, st["path"])
    X = synth.integer_points(600, 96, 200, 3)
    _, _, st = knng.build(dev(X), 10, 1.0, 0.001, 3, 3, path="auto")
    assert st["path"] == knng.PATH_MFMA_BF16X3 and st["planes"] == 1


@I8_OFF
def test_integer_form_selection(knng):
    """AUTO takes the integer form only for qualifying input; an explicit
    request on other input is refused at create."""
    base = synth.integer_points(300, 70, 255, 9)
    _, _, st = knng.build(dev(base), 8, max_iters=2, path="auto")
    assert st["path"] == knng.PATH_MFMA_I8
    wide = base.copy()
    wide[5, 5] = 256.0                      # span 256
    frac = base.copy()
    frac[7, 3] = 0.5                        # not an integer
    big = base + np.float32(2 ** 24)        # span fine, magnitude above 2^24
    for X in (wide, frac, big):
        _, _, st = knng.build(dev(X), 8, max_iters=2, path="auto")
        assert st["path"] == knng.PATH_MFMA
        with pytest.raises(knng.KnngError) as e:
            knng.build(dev(X), 8, max_iters=2, path="mfma_i8")
        assert e.value.status == 1
    _, _, st = knng.build(dev(base), 8, max_iters=2, path="auto", precision="bf16")
    assert st["path"] == knng.PATH_MFMA
    _, _, st = knng.build(dev(base[:, :8]), 8, max_iters=2, path="auto")
    assert st["path"] == knng.PATH_VALU


def test_init_matches_oracle(knng):
    X, p = synth.workload("gauss2k_d8")
    ctx = knng.Context(dev(X), 10, seed=0)
    ctx.init()
    g = ctx.export()
    ref = oracle.init(X, 10, 0)
    check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), ref.ids, ref.dists, rel=0.0)
    assert np.array_equal(np.sort(g.ids.cpu().numpy(), 1), np.sort(ref.ids, 1))
    assert (g.flags.cpu().numpy() == 1).all()


@pytest.mark.parametrize("rho", [1.0, 0.5, 0.25])
def test_sample_sets_match_oracle(knng, rho):
    """Sampled new/old sets are integer-exact, for every t of an oracle trajectory."""
    X, p = synth.workload("gauss2k_d8", N=1500)
    K = 10
    C = oracle.cap(K, rho)
    r = oracle.build_graph(X, K, rho, 0.0, 5, 7, keep_states=True)
    for s in r.states[:-1]:
        ctx = knng.Context(dev(X), K, rho=rho, seed=7)
        ctx.load(torch.from_numpy(s.ids), torch.from_numpy(s.flags), s.t)
        ctx.iterate()
        nw, od, cnt = (a.cpu().numpy() for a in ctx.samples())
        sm = oracle.sample(s, K, C, 7, s.t + 1)
        for u in range(X.shape[0]):
            a, b = cnt[u]
            assert list(nw[u, :a]) == list(sm.cnew[u]), (s.t, u)
            assert list(od[u, :b]) == list(sm.cold[u]), (s.t, u)
        ctx.close()


def test_step_parity_gauss2k(knng):
    """Load the oracle's G_t, run one GPU iteration, compare with the oracle's G_{t+1}."""
    X, p = synth.workload("gauss2k_d8")
    K = p["K"]
    r = oracle.build_graph(X, K, p["rho"], p["delta"], p["max_iters"], p["seed"], keep_states=True)
    for s, nxt, e, c in zip(r.states[:-1], r.states[1:], r.evals, r.changes):
        ctx = knng.Context(dev(X), K, rho=p["rho"], seed=p["seed"])
        ctx.load(torch.from_numpy(s.ids), torch.from_numpy(s.flags), s.t)
        eg, cg = ctx.iterate()
        assert eg == e
        g = ctx.export()
        check_rows(X, g.ids.cpu().numpy(), g.dists.cpu().numpy(), nxt.ids, nxt.dists)
        ctx.close()


def test_build_gauss2k_parity_and_recall(knng):
    X, p = synth.workload("gauss2k_d8")
    ref = oracle.build_graph(X, p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"])
    ids, dists, st = knng.build(dev(X), p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"])
    ids = ids.cpu().numpy()
    res = check_rows(X, ids, dists.cpu().numpy(), ref.ids, ref.dists)
    assert res["exact_rows"] >= X.shape[0] - 2
    ei, ed = oracle.bruteforce(X, p["K"])
    assert oracle.recall(X, ids, ed) >= 0.99
    assert st["converged"]


def test_complete_graph_N_is_K_plus_1(knng):
    X = synth.integer_points(17, 4, 9, 3)
    st = exact_build(knng, X, 16, 1.0, 0.001, 5, 3)
    assert st["iters"] == 1 and st["changes"] == [0]


def test_identical_points_hubs(knng):
    """All points equal: pure id tie-break; lists collapse onto the smallest ids,
    whose reverse pools grow past the LDS stage (radix prefilter path)."""
    X = np.full((3000, 5), 1.5, np.float32)
    exact_build(knng, X, 12, 1.0, 0.0, 6, 9)


def test_duplicate_points_and_small_K(knng):
    rng = np.random.default_rng(5)
    base = synth.integer_points(300, 6, 3, 5)
    X = base[rng.integers(0, 300, 1200)]
    exact_build(knng, X, 1, 1.0, 0.0, 8, 2)
    exact_build(knng, X, 9, 0.05, 0.0, 8, 2)


@pytest.mark.parametrize("path,N,d,K,rho,hi,seed", [
    ("valu", 400, 4, 64, 1.0, 50, 8),
    ("valu", 300, 3, 63, 1.0, 6, 12),
    ("mfma", 500, 64, 64, 0.5, 7, 13),
    ("bf16x3", 500, 64, 64, 0.5, 7, 14),
])
def test_max_K(knng, path, N, d, K, rho, hi, seed):
    """K = 63 and 64 leave (almost) no spare lane in the merge's 64-wide fold: a
    pair proposed again (by another owner, or after its id entered from an
    earlier chunk) must not cost the list an entry."""
    exact_build(knng, synth.integer_points(N, d, hi, seed), K, rho, 0.001, 6, seed, path=path)


@pytest.mark.parametrize("path,N,d,K,rho,hi,seed", [
    ("valu", 500, 2, 3, 1.0, 6, 21),
    ("valu", 500, 2, 2, 1.0, 6, 22),
    ("valu", 600, 2, 16, 1.0, 5, 23),
    ("valu", 600, 2, 17, 1.0, 5, 24),
    ("valu", 700, 3, 16, 0.5, 4, 25),
    ("bf16x3", 500, 40, 16, 1.0, 3, 26),
])
def test_merge_row_boundary(knng, path, N, d, K, rho, hi, seed):
    """Lists of up to 16 entries are merged four to a wave, one per 16-lane
    row; K = 2 and 3 leave most of a row empty, K = 16 fills it (no spare lane
    for a repeated proposal), K = 17 takes one wave per target. Small integer
    coordinates make many equal distances and many pairs proposed by several
    owners."""
    exact_build(knng, synth.integer_points(N, d, hi, seed), K, rho, 0.001, 8, seed, path=path)


@pytest.mark.parametrize("T", [1, 2, 3])
@pytest.mark.parametrize("path", ["valu", "bf16x3"])
def test_iteration_cap(knng, T, path):
    """delta = 0 never stops early here: the build runs exactly T iterations
    (the iteration enqueued ahead of the host's decision is never issued
    past T) and equals the oracle's T-iteration graph."""
    X = synth.integer_points(700, 64, 9, 21)
    ref = oracle.build_graph(X, 10, 1.0, 0.0, T, 21)
    assert ref.iters == T and ref.changes[-1] > 0
    ids, dists, st = knng.build(dev(X), 10, 1.0, 0.0, T, 21, path=path)
    assert st["iters"] == T and not st["converged"]
    assert st["evals"] == ref.evals.tolist() and st["changes"] == ref.changes.tolist()
    assert np.array_equal(ids.cpu().numpy(), ref.ids)
    assert np.array_equal(dists.cpu().numpy().astype(np.float64), ref.dists)


def test_zero_iterations_returns_init(knng):
    X, _ = synth.workload("gauss2k_d8", N=500)
    ids, dists, st = knng.build(dev(X), 10, 1.0, 0.001, 0, 4)
    ref = oracle.init(X, 10, 4)
    assert st["iters"] == 0
    assert np.array_equal(np.sort(ids.cpu().numpy(), 1), np.sort(ref.ids, 1))


def test_nonfinite_input_rejected(knng):
    X = synth.integer_points(100, 4, 5, 1)
    X[7, 2] = np.nan
    with pytest.raises(knng.KnngError) as e:
        knng.build(dev(X), 5)
    assert e.value.status == 1
    X[7, 2] = np.inf
    with pytest.raises(knng.KnngError):
        knng.build(dev(X), 5)


def test_load_rejects_bad_rows(knng):
    X = synth.integer_points(50, 3, 5, 1)
    ctx = knng.Context(dev(X), 4)
    ids = np.tile(np.arange(1, 5, dtype=np.int32), (50, 1))
    ids[1] = [0, 2, 3, 4]
    ids[2] = [0, 1, 3, 4]
    ids[3] = [0, 1, 2, 4]
    ids[4] = [0, 1, 2, 3]
    flags = np.ones((50, 4), np.uint8)
    ctx.load(torch.from_numpy(ids), torch.from_numpy(flags), 0)  # valid
    bad = ids.copy()
    bad[9, 0] = 9   # self
    with pytest.raises(knng.KnngError):
        ctx.load(torch.from_numpy(bad), torch.from_numpy(flags), 0)
    bad = ids.copy()
    bad[9, 1] = bad[9, 0]   # duplicate
    with pytest.raises(knng.KnngError):
        ctx.load(torch.from_numpy(bad), torch.from_numpy(flags), 0)


def test_deterministic_repeat(knng):
    X, p = synth.workload("gauss2k_d8")
    a = knng.build(dev(X), 10, 1.0, 0.001, 20, 0)
    b = knng.build(dev(X), 10, 1.0, 0.001, 20, 0)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert a[2]["evals"] == b[2]["evals"] and a[2]["changes"] == b[2]["changes"]


# ----------------------------------------------------------------- permutation (Sec. 3.2)

@pytest.mark.parametrize("path", ["valu", "valu3", "mfma", "bf16x3", pytest.param("mfma_i8", marks=I8_OFF)])
@pytest.mark.parametrize("tp", [1, 3])
def test_permutation_is_result_invisible_integer(knng, path, tp):
    """Reordering changes storage only: ids, distances, e_t, c_t stay bitwise
    equal, whether the permutation runs after iteration 1 or later (d = 3:
    rows and K-th keys in one record, moved together)."""
    d = 8 if path == "valu" else 3 if path == "valu3" else 72
    path = "valu" if path == "valu3" else path
    X = synth.integer_points(3000, d, 9, 21)
    a = knng.build(dev(X), 12, 0.8, 0.001, 15, 5, reorder=False, path=path)
    b = knng.build(dev(X), 12, 0.8, 0.001, 15, 5, reorder=tp, path=path)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert a[2]["evals"] == b[2]["evals"] and a[2]["changes"] == b[2]["changes"]
    assert b[2]["reorder_ms"] > 0
    st = exact_build(knng, X, 12, 0.8, 0.001, 15, 5, path=path, reorder=tp)
    assert st["iters"] == a[2]["iters"]


def test_permutation_is_result_invisible_gauss2k(knng):
    X, p = synth.workload("gauss2k_d8")
    a = knng.build(dev(X), p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"], reorder=False)
    b = knng.build(dev(X), p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"], reorder=True)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_permutation_order_and_cluster_purity(knng):
    """The order is a permutation; on data satisfying the clustered assumption
    (Sec. 3.2) each cluster ends up in (nearly) one contiguous run of
    positions, in contrast with the random input order. Fig. 4 tracks the
    same property as cluster fractions in sliding windows."""
    X, lab = synth.clustered_labels(16384, 8, 8, 3)
    ctx = knng.Context(dev(X), 20, rho=1.0, seed=1, reorder=True)
    ctx.init()
    ctx.iterate()
    ctx.iterate()
    order = ctx.order().cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(16384))
    seq = lab[order]
    changes = int((seq[1:] != seq[:-1]).sum())
    assert changes <= 64, changes                      # random order: ~14000
    for c in range(8):
        idx = np.nonzero(seq == c)[0]
        runs = np.split(idx, np.nonzero(np.diff(idx) != 1)[0] + 1)
        assert max(len(r) for r in runs) >= 0.9 * len(idx)
    ctx.close()


# ----------------------------------------------------------------- precision form (BF16 screen + FP32 rescore)

@pytest.mark.parametrize("N,d,K,rho,hi,seed", [
    (700, 64, 10, 1.0, 9, 1),
    (900, 130, 16, 0.5, 200, 3),
])
def test_bf16_screen_integer_bitwise(knng, N, d, K, rho, hi, seed):
    """Integers <= 256 are exact in BF16 and every sum is exact in FP32: the
    screened form must reproduce the oracle bit for bit."""
    X = synth.integer_points(N, d, hi, seed)
    ref = oracle.build_graph(X, K, rho, 0.001, 15, seed)
    ids, dists, st = knng.build(dev(X), K, rho, 0.001, 15, seed, precision="bf16")
    assert st["precision"] == 1
    assert st["evals"] == ref.evals.tolist() and st["changes"] == ref.changes.tolist()
    assert np.array_equal(ids.cpu().numpy(), ref.ids)
    assert np.array_equal(dists.cpu().numpy().astype(np.float64), ref.dists)
    assert all(0 < r <= 2 * e for r, e in zip(st["rescored"], st["evals"]) if e)


def test_bf16_screen_image_like_bitwise(knng):
    X = synth.image_like(2500, 1)
    ref = oracle.build_graph(X, 20, 1.0, 0.001, 30, 1)
    ids, dists, st = knng.build(dev(X), 20, 1.0, 0.001, 30, 1, precision="bf16")
    assert np.array_equal(ids.cpu().numpy(), ref.ids)
    assert st["changes"] == ref.changes.tolist()


def test_bf16_screen_continuous_parity(knng):
    """Anisotropic clusters (the precision workload's shape, N=3000): tie-aware
    parity with the FP64 oracle, stored distances within the FP32 direct-form
    bound, and the screen passes far fewer pairs than it evaluates late on."""
    X = synth.anisotropic_clusters(3000, 960, 3, 20)
    K, rho = 20, 0.5
    ref = oracle.build_graph(X, K, rho, 0.001, 30, 3)
    ids, dists, st = knng.build(dev(X), K, rho, 0.001, 30, 3, precision="bf16")
    res = check_rows(X, ids.cpu().numpy(), dists.cpu().numpy(), ref.ids, ref.dists, dpad=960, gram=False)
    assert res["exact_rows"] >= 3000 - 10
    # stored values: 32-dimension chunk sums in FP32 added into FP64, rounded
    # once: at most 13 u relative to the distance, whatever d
    D64 = oracle.list_dists(X, ids.cpu().numpy())
    err = np.abs(dists.cpu().numpy().astype(np.float64) - D64)
    assert (err <= 13 * 2.0 ** -24 * D64).all(), float((err / np.maximum(D64, 1e-300)).max())
    ei, ed = oracle.bruteforce(X, K)
    assert oracle.recall(X, ids.cpu().numpy(), ed) >= 0.99
    late = [r / (2 * e) for r, e in zip(st["rescored"], st["evals"]) if e][-3:]
    assert min(late) < 0.5


def test_bf16_screen_with_permutation(knng):
    X = synth.anisotropic_clusters(2000, 192, 5, 12)
    a = knng.build(dev(X), 12, 0.5, 0.001, 20, 5, precision="bf16", reorder=False)
    b = knng.build(dev(X), 12, 0.5, 0.001, 20, 5, precision="bf16", reorder=True)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ----------------------------------------------------------------- block-asynchronous iteration

@pytest.mark.parametrize("path,d", [("valu", 8), ("valu", 3), ("bf16x3", 72), ("mfma", 72)])
@pytest.mark.parametrize("B,reorder", [(4, 0), (16, 0), (5, 2)])
def test_block_async_integer_bitwise(knng, path, d, B, reorder):
    """Block-asynchronous builds (blocks of consecutive owner ids in order,
    each sampling from the graph the earlier blocks left) equal the oracle's
    block mode bit for bit on integer data: graph, e_t, c_t and the iteration
    count, also with the permutation running between iterations (blocks stay
    defined on original ids)."""
    X = synth.integer_points(1500, d, 9, 31)
    ref = oracle.build_graph(X, 12, 0.8, 0.001, 15, 5, blocks=B)
    ids, dists, st = knng.build(dev(X), 12, 0.8, 0.001, 15, 5, path=path, reorder=reorder, blocks=B)
    assert st["iters"] == ref.iters
    assert st["evals"] == ref.evals.tolist() and st["changes"] == ref.changes.tolist()
    assert np.array_equal(ids.cpu().numpy(), ref.ids)
    assert np.array_equal(dists.cpu().numpy().astype(np.float64), ref.dists)
    sync = oracle.build_graph(X, 12, 0.8, 0.001, 15, 5)
    assert sync.evals.tolist() != ref.evals.tolist()   # the blocks do change the trajectory


@pytest.mark.parametrize("sampling", ["weighted", "turbo"])
def test_block_async_continuous_build(knng, sampling):
    """Continuous data (the Gaussian mixture far from the origin, split form
    with FP64 accumulation), block-asynchronous builds: inside one iteration
    a near-tie that FP32 decides otherwise than FP64 in an early block changes
    what the later blocks sample, so the GPU is compared with the oracle's
    block-mode build over the trajectory: rows valid and sorted, stored
    distances within the bound, the evaluation counts within 1% (200 in the
    last, small iterations; the total within 0.5%), and the recall within
    0.005 of the oracle's."""
    X = synth.gaussian_mixture(3000, 96, 10, 10)
    K, rho, seed, B = 16, 1.0, 10, 6
    ref = oracle.build_graph(X, K, rho, 0.001, 30, seed, sampling=sampling, blocks=B)
    ids, dists, st = knng.build(dev(X), K, rho, 0.001, 30, seed, path="bf16x3", sampling=sampling, blocks=B)
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    D64, bound = fp32_bound(X, ids, 96, True, accurate=True)
    assert (np.abs(dists.astype(np.float64) - D64) <= bound).all()
    assert all(len(set(r.tolist())) == K for r in ids)
    assert not (ids == np.arange(X.shape[0])[:, None]).any()
    assert ((dists[:, 1:] > dists[:, :-1]) | ((dists[:, 1:] == dists[:, :-1]) & (ids[:, 1:] > ids[:, :-1]))).all()
    n = min(len(st["evals"]), len(ref.evals))
    assert abs(len(st["evals"]) - len(ref.evals)) <= 1
    assert np.allclose(st["evals"][:n], ref.evals[:n], rtol=0.01, atol=200)
    assert abs(sum(st["evals"]) - int(ref.evals.sum())) <= 0.005 * int(ref.evals.sum())
    _, ed = oracle.bruteforce(X, K)
    assert oracle.recall(X, ids, ed) >= oracle.recall(X, ref.ids, ed) - 0.005


def test_block_async_one_block_is_synchronous(knng):
    X, p = synth.workload("gauss2k_d8")
    a = knng.build(dev(X), p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"], blocks=0)
    b = knng.build(dev(X), p["K"], p["rho"], p["delta"], p["max_iters"], p["seed"], blocks=1)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2]["evals"] == b[2]["evals"]


# ----------------------------------------------------------------- inputs smaller than one workgroup per XCD

@pytest.mark.parametrize("N", [2, 5, 13, 28, 33])
@pytest.mark.parametrize("path,d", [("valu", 3), ("mfma", 40), ("bf16x3", 40)])
def test_tiny_inputs_bitwise(knng, N, path, d):
    """A few dozen points give fewer join workgroups than XCDs: every owner
    must still be joined (graph, e_t and c_t equal the oracle's)."""
    K = min(4, N - 1)
    exact_build(knng, synth.integer_points(N, d, 7, 40 + N), K, 1.0, 0.001, 10, 40 + N, path=path)


@pytest.mark.parametrize("N", [3, 20])
def test_tiny_inputs_precision_form(knng, N):
    X = synth.integer_points(N, 40, 7, 50 + N)
    K = min(4, N - 1)
    ref = oracle.build_graph(X, K, 1.0, 0.001, 10, 50 + N)
    ids, dists, st = knng.build(dev(X), K, 1.0, 0.001, 10, 50 + N, precision="bf16")
    assert st["evals"] == ref.evals.tolist() and st["changes"] == ref.changes.tolist()
    assert np.array_equal(ids.cpu().numpy(), ref.ids)
    assert np.array_equal(dists.cpu().numpy().astype(np.float64), ref.dists)


# ----------------------------------------------------------------- resume from an exported state

@pytest.mark.parametrize("path,gen", [("bf16x3", "aniso"), ("valu", "gauss"), ("valu", "gauss3"),
                                      ("mfma", "gauss"), ("bf16x3", "aniso_bf16")])
def test_resume_from_export_is_bitwise(knng, path, gen):
    """A state exported after t iterations and loaded with its distances into
    a new context continues exactly as the exporting build (continuous data:
    the keys are not recomputed): e_t, c_t and the final graph bit for bit."""
    if gen.startswith("aniso"):
        X = synth.anisotropic_clusters(1500, 200, 3, 12)
    else:
        X = synth.gaussian_mixture(1500, 3 if gen == "gauss3" else 16 if path == "valu" else 64, 12, 4)
    prec = "bf16" if gen.endswith("bf16") else "fp32"
    if prec == "bf16":
        path = "auto"
    K, rho, seed = 12, 0.8, 9
    a = knng.Context(dev(X), K, rho, 0.001, 30, seed, path=path, precision=prec)
    a.init()
    for _ in range(3):
        a.iterate()
    g = a.export()
    b = knng.Context(dev(X), K, rho, 0.001, 30, seed, path=path, precision=prec)
    b.load(g.ids, g.flags, 3, dists=g.dists)
    gb = b.export()
    assert torch.equal(g.ids, gb.ids) and torch.equal(g.dists, gb.dists) and torch.equal(g.flags, gb.flags)
    for _ in range(4):
        assert a.iterate() == b.iterate()
    ea, eb = a.export(), b.export()
    assert torch.equal(ea.ids, eb.ids) and torch.equal(ea.dists, eb.dists) and torch.equal(ea.flags, eb.flags)
    a.close()
    b.close()


def test_load_rejects_bad_distances(knng):
    X = synth.gaussian_mixture(300, 8, 4, 1)
    a = knng.Context(dev(X), 6, 1.0, 0.001, 10, 1, path="valu")
    a.init()
    g = a.export()
    bad = g.dists.clone()
    bad[5, 2] = -1.0
    b = knng.Context(dev(X), 6, 1.0, 0.001, 10, 1, path="valu")
    with pytest.raises(Exception):
        b.load(g.ids, g.flags, 0, dists=bad)
    bad[5, 2] = float("nan")
    with pytest.raises(Exception):
        b.load(g.ids, g.flags, 0, dists=bad)
    b.load(g.ids, g.flags, 0, dists=g.dists)
    a.close()
    b.close()
