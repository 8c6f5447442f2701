"""GPU parity of the two field options against the oracle: the map read by
nearest-node lookup (Section "Simulation", item 3) and the field evaluated
at every RK4 stage position (box lookup and map at the stage point).

Both add decisions that the (volume, bin, cell) trace does not record: which
node is nearest, and which box holds a stage point.  The oracle folds their
margins (distance to a mid-plane between nodes, to a box face or to the map's
edge, at every point where the field is read) into each muon's minimum
margin, so these tests use the whole-trajectory tie rule, with a looser bound
on the fraction of tie muons for the long shield paths (a node choice is a
decision at every step inside the map)."""
import dataclasses

import numpy as np
import pytest

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


def _with(wl, **kw):
    return dataclasses.replace(wl, run=dataclasses.replace(wl.run, **kw))


@pytest.mark.parametrize("interp,stage", [(1, 0), (0, 1), (1, 1)],
                         ids=["nearest", "stages", "nearest+stages"])
def test_shield_field_modes(interp, stage):
    wl = _with(W.make_workload("shield", n_muons=2000), interp=interp, stage_field=stage)
    n = len(wl.muons)
    o = oracle_run(wl, np.arange(n), trace_steps=1600)
    g = gpu_run(wl, trace_steps=1600, n_trace=300)
    s = compare(g, o, trace_rows=300, max_tie_frac=0.05,
                label=f"shield interp={interp} stages={stage}", **map_deltas(wl))
    print("shield", interp, stage, s)
    gp = gpu_run(wl, mode="persistent")
    for k in ("state", "status", "n_steps", "volume"):
        assert np.array_equal(g[k], gp[k]), k
    # the option changes the transport (same random streams, different field)
    base = gpu_run(W.make_workload("shield", n_muons=2000))
    assert not np.array_equal(base["state"], g["state"])


@pytest.mark.parametrize("name,n", [("block", 20_011), ("scan", 3000)])
def test_stage_field_box_geometries(name, n):
    """Uniform box fields: stage points that cross a box face (the entry face
    at z = 0, the slab faces of the 8-magnet scan) take the neighbour's field."""
    wl = _with(W.make_workload(name, n_muons=n, **({"n_variants": 2} if name == "scan" else {})),
               stage_field=1)
    g = gpu_run(wl, trace_steps=260, n_trace=1000)
    for v in range(wl.run.n_variants):
        o = oracle_run(wl, np.arange(n), variant=v, trace_steps=260)
        sel = np.arange(v * n, (v + 1) * n)
        # lanes 0..999 (variant 0) carry a per-step trace
        s = compare(g, o, sel=sel, trace_rows=1000 if v == 0 else 0,
                    label=f"{name} stages v={v}")
        print(name, "stages", v, s)


@pytest.mark.parametrize("interp", [0, 1], ids=["trilinear", "nearest"])
@pytest.mark.parametrize("stage", [0, 1], ids=["held", "stages"])
def test_uniform_map_equals_uniform_box_field(interp, stage):
    """A map whose every node holds the same field B gives B itself at every
    point inside it: the cell polynomial's non-constant coefficients are
    exactly zero and its constant one is B, and the nearest node is B.  So
    transport with that map and no box field equals, bit for bit, transport
    with the uniform box field B and no map (every muon stays inside the
    map: the world bounds lie within it)."""
    B = (0.3, 1.5, -0.2)
    box = [(-5.0, 5.0, -5.0, 5.0, 0.0, 20.0)]
    world = (4.0, 4.0, 15.0)
    rng = np.random.default_rng(5)
    n = 4000
    mu = CU.muons(rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), 0.0,
                  rng.normal(0.0, 0.5, n), rng.normal(0.0, 0.5, n), rng.uniform(5.0, 50.0, n),
                  rng.choice([-1, 1], n))
    nx, ny, nz = 11, 7, 23
    nodes = np.empty((nz, ny, nx, 3), np.float32)
    nodes[...] = np.asarray(B, np.float32)
    fmap = W.FieldMap(lo=np.array([-5.0, -5.0, -1.0]), hi=np.array([5.0, 5.0, 21.0]), b=nodes)
    hist = CU.flat_histograms()
    with_box = CU.workload(hist, CU.geometry(box, [0], b_box=[B], world=world), mu,
                           interp=interp, stage_field=stage)
    with_map = CU.workload(hist, CU.geometry(box, [0], world=world), mu, field=fmap,
                           interp=interp, stage_field=stage)
    a = gpu_run(with_box)
    b = gpu_run(with_map)
    for k in ("state", "status", "n_steps", "volume"):
        assert np.array_equal(a[k], b[k]), k
    # the field bends the tracks: they differ from a run without any field
    c = gpu_run(CU.workload(hist, CU.geometry(box, [0], world=world), mu))
    assert not np.array_equal(a["state"], c["state"])


def test_field_modes_rejected_with_checkpoints():
    import torch
    from paper_2512_10520_amd import api
    wl = W.make_workload("diff", n_muons=64)
    api.load_workload(wl)
    dm = api.DeviceMuons.from_host(wl.muons)
    sc = torch.ones((1, wl.geom.n_mag), dtype=torch.float32, device="cuda")
    for kw in ({"interp": "nearest"}, {"stage_field": True}):
        spec = api.RunSpec.from_workload(wl, **kw)
        with pytest.raises(RuntimeError, match="differentiable form"):
            api.propagate(dm, spec, scales=sc, ckpt=True)
