"""The C-ABI library loads and exports every symbol its header declares;
host-side validation rejects bad arguments without touching a GPU."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2112_06630_amd", "libknng.so")
HDR = os.path.join(ROOT, "include", "knng.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libknng.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(knng_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported(lib):
    names = declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_package_binding_loads():
    import paper_2112_06630_amd as knng
    assert knng.lib is not None
    assert os.path.samefile(knng.LIB_PATH, LIB)


def _params(**kw):
    import paper_2112_06630_amd as knng
    base = dict(K=10, rho=1.0, delta=0.001, max_iters=10, seed=0)
    base.update(kw)
    return knng.make_params(**base)


@pytest.mark.parametrize("N,d,kw,msg", [
    (100, 8, dict(K=0), "K must"),
    (100, 8, dict(K=65), "K must"),
    (10, 8, dict(K=10), "N - 1"),
    (100, 0, dict(), "d must"),
    (1, 8, dict(K=1), "N must"),
    (100, 8, dict(rho=0.0), "rho"),
    (100, 8, dict(rho=1.5), "rho"),
    (100, 8, dict(delta=-1.0), "delta"),
    (100, 8, dict(max_iters=-1), "max_iters"),
    (100, 8, dict(max_iters=65), "max_iters"),
    (100, 784, dict(K=64, rho=1.0, path="mfma"), "MFMA"),
    (100, 784, dict(path=5), "unknown path"),
    (100, 784, dict(path="bf16x3", precision="bf16"), "FP32 MFMA"),
    (100, 784, dict(K=64, rho=1.0, path="bf16x3"), "MFMA"),
    (100, 784, dict(path="mfma_i8"), "not available"),
    (100, 8, dict(sampling=2), "unknown sampling"),
    (100, 8, dict(reorder=-1), "reorder"),
    (100, 8, dict(blocks=-1), "blocks"),
    (100, 8, dict(blocks=101), "blocks"),
    (100, 8, dict(reorder=65), "reorder"),
])
def test_workspace_query_rejects(N, d, kw, msg):
    import paper_2112_06630_amd as knng
    with pytest.raises(knng.KnngError) as e:
        knng.workspace_bytes(N, d, _params(**kw))
    assert msg in str(e.value)


def test_create_rejects_before_device_work():
    """Invalid params or a short workspace fail before any HIP call."""
    import paper_2112_06630_amd as knng
    L = knng.lib
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    p = _params(K=0)
    assert L.knng_create(ctypes.byref(h), fake, 100, 8, ctypes.byref(p), fake, 1 << 30, None) == knng.EINVAL
    p = _params()
    need = knng.workspace_bytes(100, 8, p)
    assert L.knng_create(ctypes.byref(h), fake, 100, 8, ctypes.byref(p), fake, need - 1, None) == knng.ENOMEM
    assert b"workspace too small" in L.knng_last_error()
    assert L.knng_create(ctypes.byref(h), None, 100, 8, ctypes.byref(p), fake, need, None) == knng.EINVAL
    assert L.knng_build(fake, 100, 8, ctypes.byref(p), None, None, fake, need, None, None) == knng.EINVAL


def test_sample_cap_matches_oracle(oracle_lib):
    import paper_2112_06630_amd as knng
    for K in (1, 2, 7, 10, 15, 20, 64):
        for rho in (0.01, 0.3, 0.5, 0.77, 1.0):
            assert knng.sample_cap(K, rho) == oracle.cap(K, rho)


def test_workspace_takes_reorder_iteration():
    """reorder = t_p >= 1 runs the permutation after iteration t_p; every t_p
    needs the same workspace (the permuted copies)."""
    a = knng_ws(_params(reorder=1))
    assert a == knng_ws(_params(reorder=3)) == knng_ws(_params(reorder=64)) > knng_ws(_params(reorder=0))


def knng_ws(p, N=1000, d=8):
    import paper_2112_06630_amd as knng
    return knng.workspace_bytes(N, d, p)


def test_workspace_grows_with_size():
    import paper_2112_06630_amd as knng
    a = knng.workspace_bytes(1000, 8, _params())
    b = knng.workspace_bytes(2000, 8, _params())
    c = knng.workspace_bytes(2000, 784, _params(K=20))
    assert 0 < a < b < c


def test_integer_form_workspace():
    """The exact integer form is withdrawn: AUTO reserves no int8 rows; at
    high d it reserves the three BF16 planes of the split form (3 * N * dp * 2
    bytes, dp = round_up(d, 32)) on top of the FP32 MFMA layout."""
    import paper_2112_06630_amd as knng
    N, d = 3000, 784
    au = knng.workspace_bytes(N, d, _params(K=20, path="auto"))
    assert au == knng.workspace_bytes(N, d, _params(K=20, path="bf16x3"))
    mf = knng.workspace_bytes(N, d, _params(K=20, path="mfma"))
    assert 0 <= au - mf - 3 * N * 800 * 2 < 256
    assert knng.workspace_bytes(N, 8, _params(path="auto")) == knng.workspace_bytes(N, 8, _params(path="valu"))


def test_header_path_values_match_binding():
    import paper_2112_06630_amd as knng
    import re
    text = open(HDR).read()
    vals = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"(KNNG_PATH_\w+)\s*=\s*(\d+)", text))
    assert vals == {"KNNG_PATH_AUTO": knng.PATH_AUTO, "KNNG_PATH_VALU": knng.PATH_VALU,
                    "KNNG_PATH_MFMA": knng.PATH_MFMA, "KNNG_PATH_MFMA_I8": knng.PATH_MFMA_I8,
                    "KNNG_PATH_MFMA_BF16X3": knng.PATH_MFMA_BF16X3}


def _header_struct_fields(name):
    """(type, field) pairs of a `typedef struct { ... } name;` in knng.h."""
    import re
    text = open(HDR).read()
    m = re.search(r"typedef struct \{([^{}]*)\} " + name + ";", text)
    assert m, name
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        toks = decl.replace("*", " * ").split()
        field = toks[-1].split("[")[0]
        out.append((" ".join(toks[:-1]), field))
    return out


@pytest.mark.parametrize("cname,pyname", [("knng_params", "Params"), ("knng_stats", "_Stats"),
                                          ("knng_dataset", "_Dataset")])
def test_binding_structs_follow_the_header(cname, pyname):
    """The ctypes mirrors of the ABI structs have the header's fields, in order."""
    import paper_2112_06630_amd as knng
    hdr = [f for _, f in _header_struct_fields(cname)]
    py = [f for f, _ in getattr(knng, pyname)._fields_]
    assert hdr == py
