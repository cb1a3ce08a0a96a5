"""Comparison helpers for GPU-vs-oracle parity (test infrastructure).

The rule: neighbour ids must equal the oracle's except at distance ties of
1e-5 relative: every id in the symmetric difference of a row must sit at the
oracle's K-th distance tau within 1e-5 * tau, and the GPU row's entries must be
in FP64 distance order except between distances equal within 1e-5 relative.
Separately, stored FP32 distances must match an FP64 recomputation within the
FP32 error bound of the formula used (Sec. 3.3 distance, direct or Gram form).
"""
import numpy as np

import oracle

U32 = 2.0 ** -24


def fp32_bound(X, ids, dpad, gram, accurate=False):
    """Bound on |D_fp32 - D_fp64| per entry.

    Direct form: each term (x-y)^2 carries <= 3u relative error and the
    four-way partial sums add <= (dpad/4 + 2) roundings, so the error is at
    most (dpad/4 + 5) * 2u * D. Gram form: the rounding of ||x||^2 + ||y||^2 and
    2 x.y (sums of dpad products) is relative to the norms, not to D. With
    FP64 accumulation per 32-dimension step (``accurate``) only the FP32
    rounding inside a step remains (at most 32 roundings of partial sums
    bounded by sum_j |x_j y_j| <= (||x||^2 + ||y||^2) / 2, twice for 2 x.y)
    plus the final rounding of D: 34u (||x||^2 + ||y||^2) + 2u D.
    """
    D64 = oracle.list_dists(X, ids)
    if not gram:
        return D64, (dpad / 4 + 5) * 2 * U32 * D64 + 1e-30
    n = (X.astype(np.float64) ** 2).sum(1)
    nn = n[:, None] + n[ids]
    if accurate:
        return D64, 34 * U32 * nn + 2 * U32 * D64 + 1e-30
    return D64, (dpad / 4 + 8) * 4 * U32 * nn + 1e-30


def check_rows(X, gids, gd, rids, rd, rel=1e-5, dpad=None, gram=False, accurate=False):
    """Returns a dict of counts (rows, tie_rows, exact_rows, worst_tie_rel:
    the largest |D(p, q) - tau| / tau over the ids in a symmetric difference,
    worst_order_rel: the largest FP64 inversion between neighbouring entries
    of a GPU row, relative); asserts the parity rule."""
    gids = np.asarray(gids)
    rids = np.asarray(rids)
    N, K = rids.shape
    dpad = dpad or ((X.shape[1] + 3) // 4 * 4)
    D64, bound = fp32_bound(X, gids, dpad, gram, accurate)
    err = np.abs(np.asarray(gd, np.float64) - D64)
    assert (err <= bound).all(), f"stored distance off by {err.max()} (bound {bound.flat[err.argmax()]})"
    same = (np.sort(gids, 1) == np.sort(rids, 1)).all(1)
    tie_rows = 0
    worst_tie = 0.0
    for p in np.nonzero(~same)[0]:
        tau = rd[p, -1]
        tol = rel * tau + 1e-12
        diff = set(gids[p].tolist()) ^ set(rids[p].tolist())
        for q in diff:
            dq = oracle.list_dists(X[[p, q]], np.array([[1], [0]], np.int32))[0, 0]
            assert abs(dq - tau) <= tol, f"row {p}: id {q} at D={dq} is not a tie of tau={tau} (rel {abs(dq - tau) / tau:.3g})"
            worst_tie = max(worst_tie, abs(dq - tau) / max(tau, 1e-300))
        tie_rows += 1
    # order: FP64 distances of the GPU row must be non-decreasing up to ties
    inv = (D64[:, :-1] - D64[:, 1:]) / np.maximum(D64[:, 1:], 1e-300)
    dec = D64[:, 1:] < D64[:, :-1] - rel * np.maximum(D64[:, 1:], 1e-300) - 1e-12
    assert not dec.any(), f"rows out of order: {np.nonzero(dec.any(1))[0][:5]} (rel {inv.max():.3g})"
    assert all(len(set(r.tolist())) == K for r in gids), "duplicate ids in a row"
    assert not (gids == np.arange(N)[:, None]).any(), "self in a row"
    return dict(rows=N, tie_rows=tie_rows, exact_rows=int(same.sum()), worst_tie_rel=worst_tie,
                worst_order_rel=float(max(0.0, inv.max())))
