"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, the ctypes mirrors match the C struct
layout, and argument validation rejects bad calls before any device work."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_2512_10520_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mt.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmt.so is not built (run __graft_entry__.build())")
    return _lib.load()


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(mt_\w+)\s*\(", txt, re.M)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    nm = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mt_\w+)$", nm, re.M))
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)


def test_struct_layout_matches_header():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"abi_layout_{os.getpid()}")
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "abi_layout.c"), "-o", exe], check=True)
    try:
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    finally:
        os.remove(exe)
    structs = {"mt_params": _lib.MtParams, "mt_muons": _lib.MtMuons, "mt_result": _lib.MtResult}
    for line in out.strip().splitlines():
        name, field, val = line.split()
        cls = structs[name]
        if field == "sizeof":
            assert C.sizeof(cls) == int(val), name
        else:
            assert getattr(cls, field).offset == int(val), (name, field)


def test_binding_constants_match_header():
    """Every MT_* integer constant the Python binding mirrors has the value
    the header defines (modes, samplers, interpolations, axes, statuses,
    error codes)."""
    txt = open(HEADER).read()
    defs = {m.group(1): int(m.group(2))
            for m in re.finditer(r"^#define\s+(MT_\w+)\s+\(?(-?\d+)\)?", txt, re.M)}
    checked = 0
    for name, val in defs.items():
        py = name if hasattr(_lib, name) else name[3:]       # MT_ST_ZMAX -> ST_ZMAX
        if hasattr(_lib, py):
            assert getattr(_lib, py) == val, name
            checked += 1
    for code, name in _lib.ERRORS.items():
        assert defs[name] == code, name
    assert {"MT_MODE_VARIANT_WAVES", "MT_SAMPLER_ALIAS", "MT_ST_INVALID"} <= set(defs)
    assert checked >= 15


def _err(L):
    return L.mt_last_error().decode()


def test_propagate_before_load_is_rejected(L):
    L.mt_release()
    p = _lib.MtParams(step_m=0.02, max_steps=10, p_min=0.1, n_variants=1)
    rc = L.mt_propagate(C.byref(p), 1, None, None, None, None)
    assert rc == -4 and "loaded" in _err(L)


def _hist_args(**over):
    edges = np.array([1.0, 2.0, 4.0])
    counts = np.ones((1, 2, 3, 3), np.uint32)
    a = dict(n_mat=1, n_pbin=2, edges=edges, n_loss=3, loss_lo=0.0, loss_hi=0.05, n_scat=3,
             scat_lo=0.0, scat_hi=0.005, counts=counts)
    a.update(over)
    return a


def _load_hist(L, a):
    e = np.ascontiguousarray(a["edges"], np.float64)
    c = np.ascontiguousarray(a["counts"], np.uint32)
    return L.mt_load_histograms(a["n_mat"], a["n_pbin"], e.ctypes.data, a["n_loss"],
                                a["loss_lo"], a["loss_hi"], a["n_scat"], a["scat_lo"],
                                a["scat_hi"], c.ctypes.data)


def test_histogram_validation(L):
    assert _load_hist(L, _hist_args(edges=np.array([1.0, 4.0, 2.0]))) == -1
    assert "ascending" in _err(L)
    assert _load_hist(L, _hist_args(edges=np.array([0.0, 1.0, 2.0]))) == -1
    assert _load_hist(L, _hist_args(loss_hi=-1.0)) == -1
    assert _load_hist(L, _hist_args(n_pbin=0)) == -1
    empty = np.ones((1, 2, 3, 3), np.uint32)
    empty[0, 1] = 0
    assert _load_hist(L, _hist_args(counts=empty)) == -3
    assert "empty" in _err(L)
    big = np.full((1, 2, 3, 3), 2 ** 31, np.uint32)
    assert _load_hist(L, _hist_args(counts=big)) == -3
    assert _load_hist(L, _hist_args(n_loss=300, n_scat=300,
                                    counts=np.ones((1, 2, 300, 300), np.uint32))) == -7
    edges = np.geomspace(1, 10, 2000)
    assert _load_hist(L, _hist_args(n_pbin=1999, edges=edges,
                                    counts=np.ones((1, 1999, 3, 3), np.uint32))) == -7


def test_geometry_and_field_validation(L):
    world = np.array([1.0, 1.0, 1.0])
    box = np.array([[0, 1, 0, 1, 1, 0]], np.float64)       # zlo > zhi
    mat = np.array([0], np.int32)
    assert L.mt_load_geometry(1, box.ctypes.data, mat.ctypes.data, None, None, 0,
                              world.ctypes.data) == -1
    box = np.array([[0, 1, 0, 1, 0, 1]], np.float64)
    mag = np.array([3], np.int32)
    assert L.mt_load_geometry(1, box.ctypes.data, mat.ctypes.data, None, mag.ctypes.data, 2,
                              world.ctypes.data) == -1
    assert "magnet" in _err(L)
    assert L.mt_load_geometry(65, box.ctypes.data, mat.ctypes.data, None, None, 0,
                              world.ctypes.data) == -7
    assert L.mt_load_geometry(1, None, mat.ctypes.data, None, None, 0, world.ctypes.data) == -1
    lo, hi = np.zeros(3), np.ones(3)
    b = np.zeros((2, 2, 1, 3), np.float32)
    assert L.mt_load_field(1, 2, 2, lo.ctypes.data, hi.ctypes.data, b.ctypes.data) == -1
    assert L.mt_load_field(2, 2, 2, hi.ctypes.data, lo.ctypes.data, b.ctypes.data) == -1
    for bad in (np.nan, np.inf, -np.inf):
        b = np.zeros((2, 2, 2, 3), np.float32)
        b[1, 0, 1, 2] = bad
        assert L.mt_load_field(2, 2, 2, lo.ctypes.data, hi.ctypes.data, b.ctypes.data) == -1
        assert "not finite" in _err(L) and "node 5, component 2" in _err(L)


def test_option_validation(L):
    for opt, bad in ((_lib.MT_OPT_GUIDE_BITS, -1), (_lib.MT_OPT_GUIDE_BITS, 17),
                     (_lib.MT_OPT_ADJOINT_BLOCK, 96), (_lib.MT_OPT_ADJOINT_BLOCK, 512),
                     (_lib.MT_OPT_ADJOINT_LDS_HISTORY, 2), (4, 8), (99, 0)):
        assert L.mt_set_option(opt, bad) == -1, (opt, bad)
    for opt, good in ((_lib.MT_OPT_GUIDE_BITS, 0), (_lib.MT_OPT_ADJOINT_BLOCK, 64),
                      (_lib.MT_OPT_ADJOINT_LDS_HISTORY, 0)):
        assert L.mt_set_option(opt, good) == 0


def test_cell_split_division_is_exact():
    """The kernels split a cell index c into (c / n_scat, c mod n_scat) with
    one high-half product: c / n_scat = floor((c + 1) m / 2^32) with
    m = floor((2^32 - 1) / n_scat), exact for every n_scat >= 1 and c < 2^16
    (the largest histogram has 2^16 cells).  Checked for all n_scat up to 1024,
    every power of two and the largest values, over every c of the largest
    histogram with that n_scat."""
    sizes = list(range(1, 1025)) + [2 ** k for k in range(11, 17)] + [65535, 40000, 32769]
    for s in sizes:
        m = np.uint64((2 ** 32 - 1) // s)
        K = max(1, 65536 // s) * s
        c = np.arange(K, dtype=np.uint64)
        il = ((c + np.uint64(1)) * m) >> np.uint64(32)
        assert np.array_equal(il, c // np.uint64(s)), s


def test_block_geometry_validation(L):
    world = np.array([1.0, 1.0, 1.0])
    mat = np.array([0], np.int32)
    sq = [0, 0, 1, 0, 1, 1, 0, 1]
    good = np.array([[0.0, 1.0] + sq + sq], np.float64)
    bad_z = np.array([[1.0, 1.0] + sq + sq], np.float64)
    bowtie = np.array([[0.0, 1.0] + [0, 0, 1, 1, 1, 0, 0, 1] + sq], np.float64)
    flipped = np.array([[0.0, 1.0] + sq + [0, 0, 0, 1, 1, 1, 1, 0]], np.float64)
    for blk, msg in ((bad_z, "z_lo"), (bowtie, "convex"), (flipped, "convex")):
        assert L.mt_load_blocks(1, blk.ctypes.data, mat.ctypes.data, None, None, 0,
                                world.ctypes.data) == -1
        assert msg in _err(L)
    assert L.mt_load_blocks(0, good.ctypes.data, mat.ctypes.data, None, None, 0,
                            world.ctypes.data) == -1
    assert L.mt_load_blocks(65, good.ctypes.data, mat.ctypes.data, None, None, 0,
                            world.ctypes.data) == -7


def test_optimal_edges_library_matches_oracle():
    """mt_optimal_edges is host code: the library's binning equals the
    oracle's on random estimators, tolerances and grids (edges are probe
    momenta, so the comparison is exact)."""
    import oracle
    from paper_2512_10520_amd import api
    rng = np.random.default_rng(17)
    for _ in range(30):
        m = int(rng.integers(2, 600))
        p = np.sort(rng.uniform(0.1, 500.0, m))
        p = np.unique(p)
        phi = np.cumsum(rng.normal(0, rng.uniform(0.001, 0.3), len(p)))
        eps = float(rng.choice([0.0, 0.01, 0.1, 1.0, 1e9]))
        assert np.array_equal(api.optimal_edges(p, phi, eps), oracle.optimal_edges(p, phi, eps))


def test_optimal_edges_validation(L):
    p = np.array([1.0, 2.0, 3.0])
    phi = np.zeros(3)
    out = np.zeros(8)
    n = C.c_int32(0)
    assert L.mt_optimal_edges(p.ctypes.data, phi.ctypes.data, 3, -1.0, out.ctypes.data, 8,
                              C.byref(n)) == -1
    bad = np.array([1.0, 1.0, 3.0])
    assert L.mt_optimal_edges(bad.ctypes.data, phi.ctypes.data, 3, 0.1, out.ctypes.data, 8,
                              C.byref(n)) == -1
    phi = np.array([0.0, 1.0, 2.0])
    assert L.mt_optimal_edges(p.ctypes.data, phi.ctypes.data, 3, 0.1, out.ctypes.data, 2,
                              C.byref(n)) == -7
    assert L.mt_optimal_edges(p.ctypes.data, phi.ctypes.data, 3, 0.1, out.ctypes.data, 8,
                              C.byref(n)) == 0 and n.value == 3
