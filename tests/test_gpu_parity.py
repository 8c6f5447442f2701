"""GPU parity: the HIP transport against the FP64 oracle on the same Philox
streams (see tests/_parity.py for the bar)."""
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


def test_tiny_full_parity_with_trace():
    wl = W.make_workload("tiny")
    n = len(wl.muons)
    g = gpu_run(wl, trace_steps=64, n_trace=n)
    o = oracle_run(wl, np.arange(n), trace_steps=64)
    s = compare(g, o, trace_rows=n, label="tiny")
    print("tiny", s)
    assert np.all(g["status"] == oracle.ST_ZMAX)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 20_011])
def test_block_prefix_parity_ragged(n):
    wl = W.make_workload("block", n_muons=n)
    nt = min(n, 1500)
    g = gpu_run(wl, trace_steps=260, n_trace=nt)
    o = oracle_run(wl, np.arange(n), trace_steps=260)
    s = compare(g, o, trace_rows=nt, label=f"block n={n}")
    print("block", n, s)


def test_block_full_size_sampled():
    """Full 10^6-muon launch; the oracle recomputes a sample muon by muon."""
    wl = W.make_workload("block")
    n = len(wl.muons)
    g = gpu_run(wl, mode="persistent")
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([[0, 1, n - 2, n - 1], rng.choice(n, 4000, replace=False)]))
    o = oracle_run(wl, idx)
    s = compare(g, o, sel=idx, label="block full")
    print("block full", s)
    # statuses occur with the expected mix: most leave through z_max, some sideways
    counts = np.bincount(g["status"], minlength=7)
    assert counts[oracle.ST_ZMAX] > 0.5 * n and counts[oracle.ST_XMAX] > 0


def test_shield_prefix_parity_plain_and_persistent():
    wl = W.make_workload("shield", n_muons=6000)
    n = len(wl.muons)
    o = oracle_run(wl, np.arange(n), trace_steps=1600)
    g = gpu_run(wl, trace_steps=1600, n_trace=500)
    s = compare(g, o, trace_rows=500, label="shield plain", **map_deltas(wl))
    gp = gpu_run(wl, mode="persistent", trace_steps=1600, n_trace=500)
    sp = compare(gp, o, trace_rows=500, label="shield persistent", **map_deltas(wl))
    print("shield", s, sp)
    for k in ("state", "status", "n_steps", "volume", "trace"):
        assert np.array_equal(g[k], gp[k]), k


@pytest.mark.parametrize("interp,stage,sampler", [(0, 0, 0), (0, 0, 1), (1, 0, 0), (0, 1, 0),
                                                   (1, 1, 0)],
                         ids=["trilinear", "alias", "nearest", "stages", "nearest+stages"])
def test_shield_decision_time_deviation(interp, stage, sampler):
    """How far the GPU state is from the oracle's at the steps where the
    decisions are taken, on the shield (field map, 3 materials, paths up to
    1500 steps) with each field option.  A launch capped at k steps stops
    every muon still running at step k with its state there, on both sides.
    Over the muons whose (volume, bin, cell) path agrees with the oracle's up
    to that step, the largest position and relative momentum deviations at
    k = 32, 96, ..., 1504 set the map workloads' tie deltas, which must be at
    least 10x them."""
    import dataclasses
    wl = W.make_workload("shield", n_muons=3000)
    wl = dataclasses.replace(wl, run=dataclasses.replace(wl.run, interp=interp,
                                                         stage_field=stage, sampler=sampler))
    n = len(wl.muons)
    steps = 1600
    g = gpu_run(wl, trace_steps=steps, n_trace=n)
    o = oracle_run(wl, np.arange(n), trace_steps=steps)
    worst_r, worst_p, n_cmp = 0.0, 0.0, 0
    for k in range(32, 1505, 64):
        capped = dataclasses.replace(wl, run=dataclasses.replace(wl.run, max_steps=k))
        gk = gpu_run(capped)
        om = oracle.propagate(capped, np.arange(n), margins=False)
        ok = ((g["n_steps"] > k) & (o.n_steps > k) &
              (g["trace"][:, :k] == o.trace[:, :k]).all(axis=(1, 2)))
        if not ok.any():
            continue
        assert np.all(om.status[ok] == oracle.ST_STEPS) and np.all(gk["status"][ok] == 5)
        dr = np.linalg.norm(gk["state"][:3, ok] - om.state[:3, ok], axis=0)
        pm = np.linalg.norm(om.state[3:, ok], axis=0)
        dp = np.linalg.norm(gk["state"][3:, ok] - om.state[3:, ok], axis=0) / pm
        worst_r, worst_p = max(worst_r, dr.max()), max(worst_p, dp.max())
        n_cmp += int(ok.sum())
    print(f"shield interp={interp} stages={stage} sampler={sampler} decision-time deviation: "
          f"{n_cmp} (muon, step) pairs, max |dr| {worst_r:.3g} m, max rel dp {worst_p:.3g}")
    assert n_cmp > 20_000
    d = map_deltas(wl)
    assert 10 * worst_r <= d["delta_pos"] and 10 * worst_p <= d["delta_p"]


def test_scan_variants_parity():
    wl = W.make_workload("scan", n_muons=3000, n_variants=4)
    n = len(wl.muons)
    g = gpu_run(wl, mode="persistent", use_graph=True)
    for v in range(4):
        o = oracle_run(wl, np.arange(n), variant=v)
        s = compare(g, o, sel=np.arange(v * n, (v + 1) * n), label=f"scan v={v}")
        print("scan", v, s)


def test_scan_variants_plain_launch():
    """The one-launch plain form of the scan (all variants of every muon, an
    even and an odd variant count) against the oracle and bitwise against the
    persistent form."""
    for v in (4, 3):
        wl = W.make_workload("scan", n_muons=2500, n_variants=v)
        n = len(wl.muons)
        g = gpu_run(wl, mode="plain")
        gp = gpu_run(wl, mode="persistent")
        for k in g:
            assert np.array_equal(g[k], gp[k]), (v, k)
        for var in range(v):
            o = oracle_run(wl, np.arange(n), variant=var)
            s = compare(g, o, sel=np.arange(var * n, (var + 1) * n), label=f"scan plain v={var}/{v}")
            print("scan plain", v, var, s)


@pytest.mark.parametrize("steps_per_pass", [7, 32, 128, 1000, 4000])
def test_compacting_passes_match_plain_bitwise(steps_per_pass):
    """The compacting form in passes of 7 (raised to the 64-pass minimum of
    32), 32, 128, 1000 and 4000 (one pass) steps gives the plain launch's
    outputs and per-step traces bit for bit on the shield, whose paths
    (up to 1500 steps) cross many pass boundaries, with tallies."""
    wl = W.make_workload("shield", n_muons=20_000, n_fill=100_000)
    tally = {"z_det": 30.0, "r_ap": 1.0, "r_scale": 0.01}
    a = gpu_run(wl, mode="plain", trace_steps=1600, n_trace=300, tally=tally)
    b = gpu_run(wl, mode="persistent", compact_every=steps_per_pass, trace_steps=1600,
                n_trace=300, tally=tally)
    for k in a:
        assert np.array_equal(a[k], b[k]), (k, steps_per_pass)


def test_persistent_matches_plain_bitwise():
    wl = W.make_workload("block", n_muons=50_000)
    a = gpu_run(wl, mode="plain")
    for blk, c in ((64, 4), (256, 16), (512, 128)):
        b = gpu_run(wl, mode="persistent", block=blk, compact_every=c)
        for k in a:
            assert np.array_equal(a[k], b[k]), (k, blk, c)


def test_run_twice_identical():
    wl = W.make_workload("shield", n_muons=4000)
    a = gpu_run(wl, mode="persistent")
    b = gpu_run(wl, mode="persistent")
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_invalid_and_degenerate_inputs():
    hist = CU.flat_histograms()
    geom = CU.geometry([[-1, 1, -1, 1, 0, 1]], [0], world=(1.0, 1.0, 1.0))
    mu = CU.muons([0.0, np.nan, 0.0, 0.0, 0.0, 2.0, 0.0],
                  0.0,
                  [-0.01, 0.0, 0.0, 0.0, 0.0, 0.0, 5.0],
                  0.0, 0.0,
                  [50.0, 50.0, 0.0, 50.0, 0.2, 50.0, 50.0],
                  [1, 1, 1, 0, 1, 1, -1])
    wl = CU.workload(hist, geom, mu, p_min=0.5, max_steps=1000)
    g = gpu_run(wl)
    o = oracle_run(wl, np.arange(len(mu)))
    assert list(g["status"]) == list(o.status)
    assert list(g["status"][1:4]) == [oracle.ST_INVALID] * 3
    assert g["status"][4] == oracle.ST_PMIN and g["status"][5] == oracle.ST_XMAX
    assert g["status"][6] == oracle.ST_ZMAX and g["n_steps"][6] == 0
    compare(g, o, label="degenerate")
    # step cap
    wl0 = CU.workload(hist, geom, mu, p_min=0.5, max_steps=0)
    g0 = gpu_run(wl0)
    assert g0["status"][0] == oracle.ST_STEPS and g0["n_steps"][0] == 0


@pytest.mark.parametrize("n_loss,n_scat", [(16, 1), (1, 16), (1, 1)])
def test_single_row_and_single_column_histograms(n_loss, n_scat):
    """Histograms with one kick bin (the cell index is the loss index), one
    loss bin (the cell index is the kick index) or a single cell: cells,
    bins and volumes step by step against the oracle."""
    rng = np.random.default_rng(n_loss * 100 + n_scat)
    counts = rng.integers(1, 40, size=(n_loss, n_scat)).astype(np.uint32)
    hist = CU.flat_histograms(n_pbin=6, n_loss=n_loss, n_scat=n_scat, counts=counts)
    geom = CU.geometry([[-1, 1, -1, 1, 0, 3]], [0], b_box=[[0.0, 1.0, 0.0]],
                       world=(1.0, 1.0, 3.0))
    n = 2000
    mu = CU.muons(rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), -0.0075,
                  rng.normal(0, 0.1, n), rng.normal(0, 0.1, n), rng.uniform(5, 200, n),
                  np.where(np.arange(n) % 2, 1, -1))
    wl = CU.workload(hist, geom, mu, max_steps=400, p_min=0.5)
    g = gpu_run(wl, trace_steps=200, n_trace=n)
    o = oracle_run(wl, np.arange(n), trace_steps=200)
    s = compare(g, o, trace_rows=n, label=f"hist {n_loss}x{n_scat}")
    print("hist", n_loss, n_scat, s)
    cells = g["trace"][:, :, 2]
    drawn = cells[cells >= 0]
    assert drawn.size > 10_000 and drawn.max() < n_loss * n_scat
    if n_loss * n_scat > 1:
        assert len(np.unique(drawn)) == n_loss * n_scat


def test_empty_launch():
    wl = W.make_workload("tiny", n_muons=0)
    g = gpu_run(wl)
    assert g["state"].shape == (6, 0)


def test_straight_line_and_helix_on_gpu():
    """Closed forms on the GPU path: no field and no material gives a straight
    line with p unchanged; a uniform field in vacuum gives a helix of radius
    p/(kappa B) with |p| conserved to 1e-6."""
    hist = CU.flat_histograms()
    mu = CU.muons([0.0, 0.1], [0.0, -0.2], [0.0, 0.0], [0.0, 0.3], [0.0, 0.1], [10.0, 5.0], [1, -1])
    geom = CU.geometry(np.zeros((0, 6)), np.zeros(0), world=(50, 50, 1e6))
    wl = CU.workload(hist, geom, mu, max_steps=500, p_min=0.1)
    g = gpu_run(wl)
    st0 = mu.stacked()
    phat = st0[3:] / np.linalg.norm(st0[3:], axis=0)
    assert np.array_equal(g["state"][3:], st0[3:])
    assert np.allclose(g["state"][:3], st0[:3] + 500 * 0.02 * phat, rtol=0, atol=1e-6)
    B = float(np.float32(1.7))
    geom = CU.geometry([[-1e5, 1e5, -1e5, 1e5, -1e5, 1e5]], [-1], b_box=[[0, B, 0]],
                       world=(1e5, 1e5, 1e6))
    mu1 = CU.muons(0.0, 0.0, 0.0, 0.0, 0.0, 10.0, 1)
    wl = CU.workload(hist, geom, mu1, max_steps=1500, p_min=0.1)
    g = gpu_run(wl)
    R = 10.0 / (0.299792458 * B)
    c = np.array([-R, 0.0])
    r = g["state"][[0, 2], 0]
    assert abs(np.linalg.norm(r - c) - R) < 1e-6 * R
    assert abs(np.linalg.norm(g["state"][3:, 0]) / 10.0 - 1) < 1e-6


def test_tallies_against_oracle():
    wl = W.make_workload("scan", n_muons=2000, n_variants=3)
    n = len(wl.muons)
    t = {"z_det": 30.0, "r_ap": 1.0, "r_scale": 0.01}
    g = gpu_run(wl, mode="persistent", use_graph=True, tally=t)
    for v in range(3):
        o = oracle_run(wl, np.arange(n), variant=v)
        tie = (o.margin_pos < 2e-5) | (o.margin_p < 2e-6)
        term = oracle.detector_loss_terms(o.state, o.status)
        zmax = (o.status == oracle.ST_ZMAX)
        x, y, z, px, py, pz = o.state
        with np.errstate(divide="ignore", invalid="ignore"):
            rr = np.hypot(x + (30 - z) * px / pz, y + (30 - z) * py / pz)
        hit = zmax & (rr < 1.0)
        # tie muons may differ; allow their count as slack
        assert abs(g["tally"][v, 0] - zmax.sum()) <= tie.sum()
        assert abs(g["tally"][v, 1] - hit.sum()) <= tie.sum() + 1
        assert abs(g["tally"][v, 2] - term.sum()) <= tie.sum() + 1e-3 * max(1.0, term.sum())


def test_graph_replays_match_eager():
    """The graph-captured persistent launch (queue reset + transport + tallies)
    replayed several times, with unrelated eager work and synchronisations
    between replays, gives the eager launch's bits every time."""
    import torch
    from paper_2512_10520_amd import api
    wl = W.make_workload("scan", n_muons=4096, n_variants=5)
    api.load_workload(wl)
    dm = api.DeviceMuons.from_host(wl.muons)
    sc = torch.from_numpy(np.ascontiguousarray(wl.run.scales, np.float32)).cuda()
    t = {"z_det": 30.0, "r_ap": 1.0, "r_scale": 0.01}
    eager = api.propagate(dm, api.RunSpec.from_workload(wl, mode="persistent"), scales=sc, tally=t)
    torch.cuda.synchronize()
    ref = {k: getattr(eager, k).cpu().numpy() for k in ("state", "status", "n_steps", "volume",
                                                        "tally")}
    spec_g = api.RunSpec.from_workload(wl, mode="persistent", use_graph=True)
    out = api.alloc_result(spec_g, len(dm), "cuda", tally=True)
    noise = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        out.state.fill_(0.0)
        out.status.fill_(-1)
        out.tally.fill_(-1.0)
        api.propagate(dm, spec_g, scales=sc, tally=t, out=out)
        noise.mul_(1.0001).add_(0.5)                        # eager work between replays
        api.propagate(dm, api.RunSpec.from_workload(wl, mode="plain"), scales=sc)
        torch.cuda.synchronize()
        for k in ref:
            assert np.array_equal(getattr(out, k).cpu().numpy(), ref[k]), (rep, k)


@pytest.mark.parametrize("name,kw", [("block", {}), ("logbins", {}),
                                     ("scan", {"n_variants": 4})])
def test_persistent_with_trace_matches_plain(name, kw):
    """The persistent kernels of the map-free workloads (asked for 5
    waves/SIMD, a few values spilled) give the plain launch's bits, per-step
    traces included."""
    wl = W.make_workload(name, n_muons=6000, **kw)
    a = gpu_run(wl, mode="plain", trace_steps=300, n_trace=400)
    b = gpu_run(wl, mode="persistent", trace_steps=300, n_trace=400)
    for k in a:
        assert np.array_equal(a[k], b[k]), (name, k)
