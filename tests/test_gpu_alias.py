"""GPU parity of the alias-method sampler (Section "The Alias Method")
against the oracle's own alias tables and draw, on the same Philox streams:
the same bar as the inverse-CDF path (tests/_parity.py), per-step cells
included, plus bitwise agreement of the plain and persistent forms."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2512_10520_amd import workloads as W
from tests._parity import compare, gpu_run, map_deltas, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2512_10520_amd import _lib
    _lib.load()


def _alias(wl):
    return dataclasses.replace(wl, run=dataclasses.replace(wl.run, sampler=1))


def test_alias_tiny_full_parity_with_trace():
    wl = _alias(W.make_workload("tiny"))
    n = len(wl.muons)
    g = gpu_run(wl, trace_steps=64, n_trace=n)
    o = oracle_run(wl, np.arange(n), trace_steps=64)
    s = compare(g, o, trace_rows=n, label="tiny alias")
    print("tiny alias", s)
    assert np.all(g["status"] == oracle.ST_ZMAX)
    # the two samplers map the same words to different cells (at 100 GeV
    # most of the mass sits in a few cells, so most draws still agree)
    c = gpu_run(W.make_workload("tiny"), trace_steps=64, n_trace=n)
    mat = g["trace"][..., 0] >= 0
    assert (c["trace"][..., 2] != g["trace"][..., 2])[mat].sum() > 1000


@pytest.mark.parametrize("n", [65, 20_011])
def test_alias_block_prefix_parity(n):
    wl = _alias(W.make_workload("block", n_muons=n))
    nt = min(n, 1500)
    g = gpu_run(wl, trace_steps=260, n_trace=nt)
    o = oracle_run(wl, np.arange(n), trace_steps=260)
    s = compare(g, o, trace_rows=nt, label=f"block alias n={n}")
    print("block alias", n, s)


def test_alias_shield_plain_and_persistent():
    wl = _alias(W.make_workload("shield", n_muons=3000))
    n = len(wl.muons)
    o = oracle_run(wl, np.arange(n), trace_steps=1600)
    g = gpu_run(wl, trace_steps=1600, n_trace=300)
    s = compare(g, o, trace_rows=300, label="shield alias", **map_deltas(wl))
    gp = gpu_run(wl, mode="persistent", trace_steps=1600, n_trace=300)
    for k in ("state", "status", "n_steps", "volume", "trace"):
        assert np.array_equal(g[k], gp[k]), k
    print("shield alias", s)


def test_alias_scan_variants_graph():
    wl = _alias(W.make_workload("scan", n_muons=2000, n_variants=3))
    n = len(wl.muons)
    g = gpu_run(wl, mode="persistent", use_graph=True)
    for v in range(3):
        o = oracle_run(wl, np.arange(n), variant=v)
        s = compare(g, o, sel=np.arange(v * n, (v + 1) * n), label=f"scan alias v={v}")
        print("scan alias", v, s)


def test_unknown_sampler_rejected():
    import ctypes as C
    from paper_2512_10520_amd import _lib, api
    wl = W.make_workload("tiny", n_muons=4)
    api.load_workload(wl)
    dm = api.DeviceMuons.from_host(wl.muons)
    spec = api.RunSpec.from_workload(wl)
    out = api.alloc_result(spec, len(dm), "cuda")
    p = api._params(spec, None)
    p.sampler = 7
    res = _lib.MtResult(out.status.data_ptr(), out.n_steps.data_ptr(), out.volume.data_ptr())
    o = _lib.MtMuons(*[out.state[a].data_ptr() for a in range(6)], None)
    i = dm.c_struct()
    L = _lib.load()
    assert L.mt_propagate(C.byref(p), len(dm), C.byref(i), C.byref(o), C.byref(res), None) == -1
    assert "sampler" in L.mt_last_error().decode()
