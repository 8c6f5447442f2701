"""GPU parity at the documented table limits: the largest histogram
(n_loss * n_scat = 65536 cells, the guide packs 16-bit cell indices; one
pattern puts three or more cells into many guide buckets, so the probe loop
runs often) with both samplers, 1024 momentum bins, and 64 overlapping boxes
/ 64 convex blocks (one 64-bit candidate mask) probed at random and on-face
points."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2512_10520_amd import workloads as W
from tests import _custom as CU
from tests._parity import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2512_10520_amd import _lib
    _lib.load()


@pytest.mark.parametrize("sampler", [0, 1], ids=["cdf", "alias"])
def test_largest_histogram_and_most_bins(sampler):
    rng = np.random.default_rng(40)
    n_pbin, nl, ns = 1024, 256, 256
    # sparse counts with long empty runs and a few heavy cells per histogram
    counts = np.zeros((1, 4, nl, ns), np.uint32)
    for i in range(4):
        c = rng.integers(0, 3, size=(nl, ns)).astype(np.uint32) * (rng.random((nl, ns)) < 0.2)
        c[rng.integers(nl, size=5), rng.integers(ns, size=5)] += rng.integers(1000, 100000, 5).astype(np.uint32)
        counts[0, i] = c
    # pattern 3: small counts everywhere, so that many guide buckets span three
    # or more cells and the draw falls through to the probe loop
    counts[0, 3] = rng.integers(0, 4, size=(nl, ns)).astype(np.uint32)
    # 1024 momentum bins reuse the 4 patterns (bin i -> pattern i % 4)
    full = np.ascontiguousarray(counts[:, np.arange(n_pbin) % 4])
    hist = W.Histograms(p_edges=W.log_edges(1.0, 1000.0, n_pbin), loss_lo=0.0, loss_hi=0.05,
                        scat_lo=0.0, scat_hi=5e-3, counts=full)
    geom = CU.geometry([[-5, 5, -5, 5, 0, 3]], [0], b_box=[[0, 1.0, 0]], world=(5.0, 5.0, 3.0))
    n = 3000
    p = np.geomspace(2.0, 900.0, n)
    mu = CU.muons(rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), -0.0075, 0.0, 0.0, p,
                  np.where(np.arange(n) % 2, 1, -1))
    wl = CU.workload(hist, geom, mu, max_steps=200, p_min=1.0, sampler=sampler)
    g = gpu_run(wl, trace_steps=200, n_trace=n)
    o = oracle_run(wl, np.arange(n), trace_steps=200)
    s = compare(g, o, trace_rows=n, label=f"limits sampler={sampler}")
    assert g["trace"][..., 2].max() > 60000           # cells near the top of the range occur
    print("limits", sampler, s)


def _probe(wl, pts):
    n = len(pts)
    mu = CU.muons(pts[:, 0], pts[:, 1], pts[:, 2], 0.0, 0.0, 10.0, 1)
    wl = dataclasses.replace(wl, muons=mu)
    g = gpu_run(wl)
    expect = np.array([oracle.lookup(wl, p) for p in pts], np.int32)
    return g["volume"], expect


def test_64_overlapping_boxes():
    rng = np.random.default_rng(41)
    lo = rng.uniform(-2, 1.5, size=(64, 3))
    hi = lo + rng.uniform(0.1, 1.5, size=(64, 3))
    boxes = np.stack([lo[:, 0], hi[:, 0], lo[:, 1], hi[:, 1], lo[:, 2], hi[:, 2]], axis=1)
    geom = CU.geometry(boxes, rng.integers(-1, 1, 64), world=(10.0, 10.0, 10.0))
    wl = CU.workload(CU.flat_histograms(), geom, CU.muons(0, 0, 0, 0, 0, 1, 1), max_steps=0,
                     p_min=0.1)
    pts = rng.uniform(-2.5, 3.5, size=(4000, 3))
    faces = boxes[rng.integers(64, size=500)]
    on = np.stack([faces[:, rng.integers(2)], rng.uniform(-2, 3, 500), faces[:, 4 + rng.integers(2)]], 1)
    got, expect = _probe(wl, np.vstack([pts, on]))
    assert np.array_equal(got, expect)
    assert len(np.unique(expect)) > 40


def test_64_convex_blocks():
    rng = np.random.default_rng(42)
    blocks = []
    for b in range(64):
        cx, cy, z0 = rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0, 8)
        r0, r1 = rng.uniform(0.3, 1.0), rng.uniform(0.3, 1.0)
        ang = rng.uniform(0, 2 * np.pi)
        quad = lambda r, a: [v for k in range(4) for v in (cx + r * np.cos(a + k * np.pi / 2),
                                                           cy + r * np.sin(a + k * np.pi / 2))]
        blocks.append([z0, z0 + rng.uniform(0.5, 2.0)] + quad(r0, ang) + quad(r1, ang + 0.3))
    geom = CU.geometry(None, rng.integers(-1, 1, 64), world=(10.0, 10.0, 20.0), poly=blocks)
    wl = CU.workload(CU.flat_histograms(), geom, CU.muons(0, 0, 0, 0, 0, 1, 1), max_steps=0,
                     p_min=0.1)
    pts = rng.uniform([-3.5, -3.5, -0.5], [3.5, 3.5, 10.5], size=(5000, 3))
    got, expect = _probe(wl, pts)
    assert np.array_equal(got, expect)
    assert len(np.unique(expect)) > 40
