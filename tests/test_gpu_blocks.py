"""GPU parity of the convex-block geometry (Section "Simulation", item 1: the
interpolated quadrilateral slice, the sign test of Eq. (1) and a spatial
grid that prunes candidates) against the oracle, which tests every block.
Same bar as the box geometry (tests/_parity.py); the oracle's margins include
the in-slice distance to every block edge and to the z faces."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2512_10520_amd import workloads as W
from tests import _custom as CU
from tests._parity import compare, gpu_run, map_deltas, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2512_10520_amd import _lib
    _lib.load()


def test_blocks_parity_plain_and_persistent():
    wl = W.make_workload("blocks", n_muons=5000)
    n = len(wl.muons)
    o = oracle_run(wl, np.arange(n), trace_steps=1600)
    g = gpu_run(wl, trace_steps=1600, n_trace=600)
    s = compare(g, o, trace_rows=600, label="blocks plain")
    gp = gpu_run(wl, mode="persistent", trace_steps=1600, n_trace=600)
    for k in ("state", "status", "n_steps", "volume", "trace"):
        assert np.array_equal(g[k], gp[k]), k
    print("blocks", s)
    # the muons visit the tapered parts: some end inside a yoke or the core
    assert np.isin(g["volume"], np.arange(40)).sum() > 0


def test_blocks_with_map_and_alias():
    """Blocks with the shield's trilinear map added and the alias sampler."""
    wl = W.make_workload("blocks", n_muons=3000)
    fmap = W.make_workload("shield", n_muons=1, n_fill=1000).field
    wl = dataclasses.replace(wl, field=fmap, run=dataclasses.replace(wl.run, sampler=1))
    n = len(wl.muons)
    o = oracle_run(wl, np.arange(n), trace_steps=1600)
    g = gpu_run(wl, trace_steps=1600, n_trace=300)
    s = compare(g, o, trace_rows=300, label="blocks map alias", **map_deltas(wl))
    print("blocks map alias", s)


def test_block_lookup_on_faces_and_overlaps():
    """Points on and next to block faces and edges, in overlapping blocks
    (lowest index wins) and outside the grid: one-step probes from chosen
    start points give the oracle's final volume exactly (zero field, no
    material, so the start point is the point looked up at the end when
    max_steps = 0)."""
    rect = [0.0, 0.0, 2.0, 0.0, 2.0, 2.0, 0.0, 2.0]
    tri_top = [0.5, 0.5, 1.5, 0.5, 1.5, 1.5, 0.5, 1.5]
    b0 = [0.0, 1.0] + rect + tri_top
    b1 = [0.5, 3.0] + [v + 1.0 for v in rect] + [v + 1.0 for v in rect]
    b2 = [1.0, 2.0] + [-3.0, -3.0, -1.0, -3.0, -1.0, -1.0, -3.0, -1.0] + \
         [-3.0, -3.0, -1.0, -3.0, -1.0, -1.0, -3.0, -1.0]
    geom = CU.geometry(None, [-1, -1, -1], world=(10.0, 10.0, 10.0), poly=[b0, b1, b2])
    rng = np.random.default_rng(3)
    pts = [[1.0, 1.0, 0.0], [1.0, 1.0, 1.0], [0.0, 0.0, 0.0], [2.0, 2.0, 0.0], [1.5, 1.5, 0.7],
           [2.5, 2.5, 0.7], [3.0, 3.0, 0.5], [3.0, 3.0, 3.0], [-1.0, -1.0, 1.5], [-3.0, -2.0, 1.0],
           [-3.0, -2.0, 2.0], [5.0, 5.0, 5.0], [-9.0, 0.0, 0.0], [0.25, 0.25, 0.5]]
    pts += list(rng.uniform([-3.5, -3.5, -0.5], [3.5, 3.5, 3.5], size=(2000, 3)))
    pts = np.array(pts)
    n = len(pts)
    mu = CU.muons(pts[:, 0], pts[:, 1], pts[:, 2], 0.0, 0.0, 10.0, 1)
    wl = CU.workload(CU.flat_histograms(), geom, mu, max_steps=0, p_min=0.1)
    g = gpu_run(wl)
    expect = [oracle.lookup(wl, p) for p in pts]
    assert np.array_equal(g["volume"], np.array(expect, np.int32))
    assert expect[4] == 0 and expect[5] == 1 and expect[6] == 1


def test_block_lookup_cache_along_paths():
    """A lane keeps the block of its previous step when its point is clear
    inside it and no lower-index block can reach into it (checked at load).
    Straight vacuum paths through overlapping, face-sharing and twisted
    blocks: the per-step volume of every muon equals the oracle's lookup
    (which tests every block, lowest index first) at every step, and the
    final volumes and states agree."""
    rect = lambda x0, x1, y0, y1: [x0, y0, x1, y0, x1, y1, x0, y1]
    blocks = [
        [0.0, 2.0] + rect(-1.0, 0.2, -1.0, 1.0) + rect(-1.0, 0.5, -1.0, 1.0),    # 0: reaches into 1
        [0.5, 2.5] + rect(0.0, 1.0, -1.0, 1.0) + rect(0.0, 1.0, -1.0, 1.0),      # 1: overlapped by 0
        [0.0, 2.5] + rect(1.0, 2.0, -1.0, 1.0) + rect(1.0, 2.0, -1.0, 1.0),      # 2: shares x = 1 with 1
        [0.0, 2.5] + rect(-2.0, -1.0, -1.0, 1.0) + [-2.0, -0.8, -1.2, -1.0, -1.0, 1.0, -2.0, 0.9],  # 3: twisted
    ]
    geom = CU.geometry(None, [-1, -1, -1, -1], world=(3.0, 3.0, 2.6), poly=blocks)
    rng = np.random.default_rng(11)
    n = 3000
    x0, y0 = rng.uniform(-2.2, 2.2, n), rng.uniform(-1.2, 1.2, n)
    px, py = rng.normal(0.0, 0.4, n), rng.normal(0.0, 0.2, n)
    mu = CU.muons(x0, y0, -0.005, px, py, 10.0, 1)
    wl = CU.workload(CU.flat_histograms(), geom, mu, max_steps=300, p_min=0.1)
    g = gpu_run(wl, trace_steps=300, n_trace=n)
    o = oracle_run(wl, np.arange(n), trace_steps=300)
    s = compare(g, o, trace_rows=n, label="block cache paths")
    print("block cache paths", s)
    vols = np.unique(g["trace"][:, :, 0])
    assert {0, 1, 2, 3} <= set(vols.tolist())


def test_blocks_reject_unsupported_forms():
    import torch
    from paper_2512_10520_amd import api
    wl = W.make_workload("blocks", n_muons=64, n_fill=1000)
    api.load_workload(wl)
    dm = api.DeviceMuons.from_host(wl.muons)
    with pytest.raises(RuntimeError, match="convex-block"):
        api.propagate(dm, api.RunSpec.from_workload(wl, stage_field=True))
    sc = torch.ones((1, wl.geom.n_mag), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="convex-block"):
        api.propagate(dm, api.RunSpec.from_workload(wl), scales=sc, ckpt=True)
