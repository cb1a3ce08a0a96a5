"""FP64 CPU oracle for synchronous, seeded NN-Descent (squared l2).

Test infrastructure only: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``. The product package never imports it.

The arithmetic lives in ``knng_oracle.c`` (plain C, FP64, OpenMP over
independent nodes); this module only marshals numpy arrays through ctypes,
plus numpy helpers for recall that follow the paper's definitions:

* Sec. 2: the exact K-NNG keeps, for every vertex, the k nearest other
  vertices; recall measures how close the NN-Descent graph is to it.
* Sec. 2: one l2 evaluation costs d subtractions, d multiplications and d-1
  additions (3d-1 flops).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knng_oracle.c")
_LIB_PATH = os.environ.get("KNNG_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))
_lib = None

NEW = 1
OLD = 0


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math so FP64 order is fixed)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, u64, u32, f64 = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                               ctypes.c_uint32, ctypes.c_double)
    lib.orc_mix64.argtypes = [u64]
    lib.orc_mix64.restype = u64
    lib.orc_hash.argtypes = [u64, u64, u64, u32, u32]
    lib.orc_hash.restype = u64
    lib.orc_cap.argtypes = [i32, f64]
    lib.orc_cap.restype = i32
    lib.orc_dist.argtypes = [P, i64, i64, i64]
    lib.orc_dist.restype = f64
    lib.orc_init.argtypes = [P, i64, i32, i32, u64, P, P, P]
    lib.orc_sample.argtypes = [P, P, i64, i32, i32, u64, i32, P, P, P, P, P, i32]
    lib.orc_join_merge.argtypes = [P, i64, i32, i32, i32, P, P, P, P, P, P, P, P, P]
    lib.orc_iterate.argtypes = [P, i64, i32, i32, i32, u64, i32, P, P, P, P, P, i32]
    lib.orc_iterate_blocks.argtypes = [P, i64, i32, i32, i32, u64, i32, i32, P, P, P, P, P, i32]
    lib.orc_dist_sum.argtypes = [P, i64, i32]
    lib.orc_dist_sum.restype = f64
    lib.orc_build.argtypes = [P, i64, i32, i32, f64, f64, i32, u64, P, P, P, P, P, P, i32]
    lib.orc_bruteforce.argtypes = [P, i64, i32, i32, P, P]
    lib.orc_bruteforce_rows.argtypes = [P, i64, i32, i32, P, i64, P, P]
    lib.orc_list_dists.argtypes = [P, i64, i32, i32, P, P]
    lib.orc_greedy_order.argtypes = [P, i64, i32, P, P]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = None
    for name in ("orc_init", "orc_sample", "orc_join_merge", "orc_iterate", "orc_iterate_blocks", "orc_build",
                 "orc_bruteforce", "orc_bruteforce_rows", "orc_list_dists", "orc_greedy_order"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(X) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be 2-D [N, d]")
    return X


def _check(rc: int, what: str):
    if rc < 0:
        raise ValueError(f"oracle {what} failed (rc={rc})")


def mix64(z: int) -> int:
    return int(_load().orc_mix64(z & 0xFFFFFFFFFFFFFFFF))


def hash64(seed: int, tag: int, t: int, a: int, b: int) -> int:
    return int(_load().orc_hash(seed, tag, t, a, b))


def cap(K: int, rho: float) -> int:
    return int(_load().orc_cap(K, rho))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later oracle calls (the results do not depend on it)."""
    _load().orc_set_num_threads(int(n))


@dataclass
class State:
    """Oracle graph state: ids/dists/flags [N, K], rows sorted by (dist, id)."""
    ids: np.ndarray
    dists: np.ndarray
    flags: np.ndarray
    t: int = 0

    def copy(self) -> "State":
        return State(self.ids.copy(), self.dists.copy(), self.flags.copy(), self.t)


def init(X, K: int, seed: int) -> State:
    X = _f32(X)
    N, d = X.shape
    ids = np.empty((N, K), np.int32)
    dists = np.empty((N, K), np.float64)
    flags = np.empty((N, K), np.uint8)
    _check(_load().orc_init(_ptr(X), N, d, K, seed, _ptr(ids), _ptr(dists), _ptr(flags)), "init")
    return State(ids, dists, flags, 0)


@dataclass
class Sample:
    cnew: list  # per node: array of sampled new member ids, sorted by (w, id)
    cold: list
    flags: np.ndarray  # flags after the new->old flip


SAMPLING = {"weighted": 0, "turbo": 1}


def _mode(sampling: str) -> int:
    if sampling not in SAMPLING:
        raise ValueError(f"sampling must be one of {sorted(SAMPLING)}")
    return SAMPLING[sampling]


def sample(state: State, K: int, C: int, seed: int, t: int, sampling: str = "weighted") -> Sample:
    """Sampling step of iteration t (Sec. 3.1): the heap rule ("weighted") or
    turbosampling ("turbo")."""
    N = state.ids.shape[0]
    cnew = np.empty((N, C), np.int32)
    cold = np.empty((N, C), np.int32)
    nnew = np.empty(N, np.int32)
    nold = np.empty(N, np.int32)
    f2 = np.empty((N, K), np.uint8)
    ids = np.ascontiguousarray(state.ids, np.int32)
    fl = np.ascontiguousarray(state.flags, np.uint8)
    _check(_load().orc_sample(_ptr(ids), _ptr(fl), N, K, C, seed, t, _ptr(cnew), _ptr(nnew),
                              _ptr(cold), _ptr(nold), _ptr(f2), _mode(sampling)), "sample")
    return Sample([cnew[u, :nnew[u]].copy() for u in range(N)],
                  [cold[u, :nold[u]].copy() for u in range(N)], f2)


def sample_arrays(state: State, K: int, C: int, seed: int, t: int, sampling: str = "weighted"):
    """The sampling step as arrays (large inputs): cnew, cold [N, C] (ids of
    the sampled members, the first nnew / nold of each row valid), nnew,
    nold [N] and the flags after the flip [N, K]."""
    N = state.ids.shape[0]
    cnew = np.full((N, C), -1, np.int32)
    cold = np.full((N, C), -1, np.int32)
    nnew = np.empty(N, np.int32)
    nold = np.empty(N, np.int32)
    f2 = np.empty((N, K), np.uint8)
    ids = np.ascontiguousarray(state.ids, np.int32)
    fl = np.ascontiguousarray(state.flags, np.uint8)
    _check(_load().orc_sample(_ptr(ids), _ptr(fl), N, K, C, seed, t, _ptr(cnew), _ptr(nnew),
                              _ptr(cold), _ptr(nold), _ptr(f2), _mode(sampling)), "sample")
    return cnew, nnew, cold, nold, f2


def join_merge(X, state: State, smp: Sample, K: int, C: int) -> tuple[State, int, int]:
    """Join and merge (Sec. 2 calculation step) of one iteration on the sampled
    sets ``smp`` of ``state`` (its flags replaced by ``smp.flags``, the flags
    after sampling). Returns (new state, e_t, c_t)."""
    X = _f32(X)
    N, d = X.shape
    s = state.copy()
    s.flags = np.ascontiguousarray(smp.flags, np.uint8).copy()
    s.ids = np.ascontiguousarray(s.ids, np.int32)
    s.dists = np.ascontiguousarray(s.dists, np.float64)
    cnew = np.zeros((N, C), np.int32)
    cold = np.zeros((N, C), np.int32)
    nnew = np.array([len(a) for a in smp.cnew], np.int32)
    nold = np.array([len(a) for a in smp.cold], np.int32)
    for u in range(N):
        cnew[u, :nnew[u]] = smp.cnew[u]
        cold[u, :nold[u]] = smp.cold[u]
    e = ctypes.c_int64(0)
    c = ctypes.c_int64(0)
    _check(_load().orc_join_merge(_ptr(X), N, d, K, C, _ptr(cnew), _ptr(nnew), _ptr(cold), _ptr(nold),
                                  _ptr(s.ids), _ptr(s.dists), _ptr(s.flags), ctypes.byref(e), ctypes.byref(c)),
           "join_merge")
    s.t += 1
    return s, int(e.value), int(c.value)


def iterate(X, state: State, K: int, C: int, seed: int,
            sampling: str = "weighted", blocks: int = 1) -> tuple[State, int, int]:
    """One iteration t = state.t + 1: synchronous (blocks = 1), or block-
    asynchronous over ``blocks`` blocks of consecutive owner ids (each block
    samples from the graph the earlier blocks left). Returns (new state, e_t, c_t)."""
    X = _f32(X)
    N, d = X.shape
    s = state.copy()
    e = ctypes.c_int64(0)
    c = ctypes.c_int64(0)
    if blocks > 1:
        _check(_load().orc_iterate_blocks(_ptr(X), N, d, K, C, seed, s.t + 1, int(blocks), _ptr(s.ids),
                                          _ptr(s.dists), _ptr(s.flags), ctypes.byref(e), ctypes.byref(c),
                                          _mode(sampling)), "iterate_blocks")
    else:
        _check(_load().orc_iterate(_ptr(X), N, d, K, C, seed, s.t + 1, _ptr(s.ids), _ptr(s.dists),
                                   _ptr(s.flags), ctypes.byref(e), ctypes.byref(c), _mode(sampling)),
               "iterate")
    s.t += 1
    return s, int(e.value), int(c.value)


@dataclass
class BuildResult:
    ids: np.ndarray
    dists: np.ndarray
    flags: np.ndarray
    iters: int
    evals: np.ndarray
    changes: np.ndarray
    dist_sum: np.ndarray
    states: list = field(default_factory=list)


def build_graph(X, K: int, rho: float, delta: float, max_iters: int, seed: int,
                keep_states: bool = False, sampling: str = "weighted", blocks: int = 1) -> BuildResult:
    """Whole build (synchronous, or block-asynchronous with ``blocks`` > 1).
    With keep_states, every G_t (t = 0..iters) is kept."""
    X = _f32(X)
    N, d = X.shape
    C = cap(K, rho)
    st = init(X, K, seed)
    states = [st.copy()] if keep_states else []
    ev, ch, ds = [], [], []
    for t in range(1, max_iters + 1):
        st, e, c = iterate(X, st, K, C, seed, sampling, blocks)
        ev.append(e)
        ch.append(c)
        ds.append(float(_load().orc_dist_sum(_ptr(st.dists), N, K)))
        if keep_states:
            states.append(st.copy())
        if c < delta * N * K:
            break
    return BuildResult(st.ids, st.dists, st.flags, st.t, np.array(ev, np.int64),
                       np.array(ch, np.int64), np.array(ds), states)


def build_graph_c(X, K: int, rho: float, delta: float, max_iters: int, seed: int,
                  sampling: str = "weighted") -> BuildResult:
    """Whole build in one C call (used for timing)."""
    X = _f32(X)
    N, d = X.shape
    ids = np.empty((N, K), np.int32)
    dists = np.empty((N, K), np.float64)
    flags = np.empty((N, K), np.uint8)
    m = max(max_iters, 1)
    ev = np.zeros(m, np.int64)
    ch = np.zeros(m, np.int64)
    ds = np.zeros(m, np.float64)
    it = _load().orc_build(_ptr(X), N, d, K, rho, delta, max_iters, seed, _ptr(ids), _ptr(dists),
                           _ptr(flags), _ptr(ev), _ptr(ch), _ptr(ds), _mode(sampling))
    _check(it, "build")
    return BuildResult(ids, dists, flags, it, ev[:it], ch[:it], ds[:it])


def bruteforce(X, K: int) -> tuple[np.ndarray, np.ndarray]:
    """Exact K-NN (FP64, self excluded, ties by id)."""
    X = _f32(X)
    N, d = X.shape
    ids = np.empty((N, K), np.int32)
    dists = np.empty((N, K), np.float64)
    _check(_load().orc_bruteforce(_ptr(X), N, d, K, _ptr(ids), _ptr(dists)), "bruteforce")
    return ids, dists


def bruteforce_rows(X, K: int, rows) -> tuple[np.ndarray, np.ndarray]:
    X = _f32(X)
    N, d = X.shape
    rows = np.ascontiguousarray(rows, np.int64)
    ids = np.empty((len(rows), K), np.int32)
    dists = np.empty((len(rows), K), np.float64)
    _check(_load().orc_bruteforce_rows(_ptr(X), N, d, K, _ptr(rows), len(rows), _ptr(ids),
                                       _ptr(dists)), "bruteforce_rows")
    return ids, dists


def greedy_order(ids) -> tuple[np.ndarray, np.ndarray]:
    """Sec. 3.2 greedy clustering heuristic on a list graph whose rows are
    sorted nearest first: returns (sigma, sigma_inv), sigma[node] = spot."""
    ids = np.ascontiguousarray(ids, np.int32)
    N, K = ids.shape
    sigma = np.empty(N, np.int32)
    inv = np.empty(N, np.int32)
    _check(_load().orc_greedy_order(_ptr(ids), N, K, _ptr(sigma), _ptr(inv)), "greedy_order")
    return sigma, inv


def list_dists(X, ids) -> np.ndarray:
    """FP64 D(p, ids[p, k]) for every entry."""
    X = _f32(X)
    N, d = X.shape
    ids = np.ascontiguousarray(ids, np.int32)
    K = ids.shape[1]
    out = np.empty(ids.shape, np.float64)
    _check(_load().orc_list_dists(_ptr(X), N, d, K, _ptr(ids), _ptr(out)), "list_dists")
    return out


def recall(X, ids, exact_dists, rows=None, rel: float = 1e-5) -> float:
    """Tie-aware recall of the found lists ``ids`` [N, K].

    A found id q of p counts as correct when D(p, q) <= tau_p * (1 + rel), with
    tau_p the exact FP64 K-th distance of p (``exact_dists[:, -1]``). With
    ``rows`` only those query rows are scored (sampled recall) and
    ``exact_dists`` holds their exact lists in the same order.
    """
    X = _f32(X)
    ids = np.asarray(ids)
    q = np.arange(ids.shape[0], dtype=np.int64) if rows is None else np.asarray(rows, np.int64)
    ids = ids[q]
    Xd = X.astype(np.float64)
    good = 0
    for s in range(0, len(q), 2048):
        qq = q[s:s + 2048]
        diff = Xd[ids[s:s + 2048]] - Xd[qq][:, None, :]
        D = np.einsum("nkd,nkd->nk", diff, diff)
        tau = np.asarray(exact_dists)[s:s + 2048, -1][:, None]
        good += int(np.count_nonzero(D <= tau * (1.0 + rel)))
    return good / ids.size


def plain_recall(found_ids, exact_ids) -> float:
    found_ids = np.asarray(found_ids)
    exact_ids = np.asarray(exact_ids)
    hit = 0
    for a, b in zip(found_ids, exact_ids):
        hit += len(np.intersect1d(a, b, assume_unique=True))
    return hit / exact_ids.size
