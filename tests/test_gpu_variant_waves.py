"""GPU: the variant-wave form (lanes holding variants of one muon share its
Philox stream; 64 variants fill a wavefront) against the one-launch plain
form, bit for bit, and against the FP64 oracle on sampled variants."""
import numpy as np
import pytest

from paper_2512_10520_amd import workloads as W
from tests._parity import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

KEYS = ("state", "status", "n_steps", "volume")


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2512_10520_amd import _lib
    _lib.load()


def _same(a, b, label):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (label, k)


def test_scan_64_variants_bitwise_and_oracle():
    """The design scan's 64 variants on a ragged muon count: every output of
    every lane equals the plain launch's, and three variants match the
    oracle."""
    wl = W.make_workload("scan", n_muons=701)
    n = len(wl.muons)
    assert wl.run.n_variants == 64
    g = gpu_run(wl, mode="variant_waves")
    _same(g, gpu_run(wl, mode="plain"), "scan 64")
    for var in (0, 37, 63):
        o = oracle_run(wl, np.arange(n), variant=var)
        s = compare(g, o, sel=np.arange(var * n, (var + 1) * n), label=f"variant waves v={var}")
        print("variant waves", var, s)


@pytest.mark.parametrize("block", [64, 192, 1024])
def test_two_groups_and_block_sizes(block):
    """128 variants (two 64-lane groups per muon) at several block sizes."""
    wl = W.make_workload("scan", n_muons=300)
    sc = np.random.default_rng(5).uniform(0.8, 1.2, size=(128, wl.geom.n_mag)).astype(np.float32)
    a = gpu_run(wl, mode="plain", n_variants=128, scales=sc)
    b = gpu_run(wl, mode="variant_waves", n_variants=128, scales=sc, block=block)
    _same(a, b, f"128 variants block {block}")


@pytest.mark.parametrize("name,sampler,interp,stage", [
    ("shield", "cdf", "trilinear", False),
    ("shield", "alias", "nearest", False),
    ("shield", "cdf", "trilinear", True),
    ("blocks", "cdf", "trilinear", False),
    ("logbins", "alias", "trilinear", False),
])
def test_kernel_variants(name, sampler, interp, stage):
    """Field map (trilinear, nearest, per-stage), alias sampler, convex
    blocks and log10 axes, 64 variants each: bitwise equal to plain."""
    import dataclasses
    wl = W.make_workload(name, n_muons=160)
    wl = dataclasses.replace(wl, run=dataclasses.replace(
        wl.run, sampler=1 if sampler == "alias" else 0, interp=1 if interp == "nearest" else 0,
        stage_field=int(stage)))
    n_mag = max(wl.geom.n_mag, 1)
    sc = np.random.default_rng(9).uniform(0.8, 1.2, size=(64, n_mag)).astype(np.float32)
    sc = sc if wl.geom.n_mag > 0 else None
    a = gpu_run(wl, mode="plain", n_variants=64, scales=sc)
    b = gpu_run(wl, mode="variant_waves", n_variants=64, scales=sc)
    _same(a, b, f"{name} {sampler} {interp} {stage}")
    if sc is None:      # identical variants: every copy of a muon ends the same way
        n = len(wl.muons)
        st = b["state"].reshape(6, 64, n)
        assert np.array_equal(st, np.broadcast_to(st[:, :1], st.shape))


def test_graph_replays_and_autotune():
    import torch
    from paper_2512_10520_amd import api
    wl = W.make_workload("scan", n_muons=2000)
    api.load_workload(wl)
    dm = api.DeviceMuons.from_host(wl.muons)
    sc = torch.from_numpy(np.ascontiguousarray(wl.run.scales, np.float32)).cuda()
    ref = api.propagate(dm, api.RunSpec.from_workload(wl, mode="plain"), scales=sc)
    torch.cuda.synchronize()
    spec = api.RunSpec.from_workload(wl, mode="variant_waves", use_graph=True)
    out = api.alloc_result(spec, len(dm), "cuda")
    for rep in range(3):
        out.state.fill_(0.0)
        out.status.fill_(-1)
        api.propagate(dm, spec, scales=sc, out=out)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(getattr(out, k), getattr(ref, k)), (rep, k)
    t = api.autotune(dm, api.RunSpec.from_workload(wl, mode="variant_waves"), scales=sc)
    assert t["block"] in (64, 128, 256, 512) and t["compact_every"] == 0 and t["ms"] > 0
    got = api.propagate(dm, api.RunSpec.from_workload(wl, mode="variant_waves"), scales=sc)
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(getattr(got, k), getattr(ref, k)), ("tuned", k)


@pytest.mark.parametrize("nv", [2, 3, 8, 12, 32, 96])
def test_other_variant_counts(nv):
    """Variant counts whose largest power-of-two divisor G is below 64 (a
    wavefront then holds 64 / G muons, G lanes sharing each random stream;
    G = 1 for 3 variants) on a muon count that leaves the last wavefront
    ragged: bitwise equal to the plain launch."""
    wl = W.make_workload("scan", n_muons=301)
    sc = np.random.default_rng(nv).uniform(0.8, 1.2, size=(nv, wl.geom.n_mag)).astype(np.float32)
    a = gpu_run(wl, mode="plain", n_variants=nv, scales=sc)
    b = gpu_run(wl, mode="variant_waves", n_variants=nv, scales=sc)
    _same(a, b, f"{nv} variants")


def test_rejected_arguments():
    """A trace and the checkpointed form are refused before any launch."""
    import torch
    from paper_2512_10520_amd import api
    wl = W.make_workload("scan", n_muons=100, n_variants=8)
    api.load_workload(wl)
    dm = api.DeviceMuons.from_host(wl.muons)
    wl64 = W.make_workload("scan", n_muons=100)
    sc64 = torch.from_numpy(np.ascontiguousarray(wl64.run.scales, np.float32)).cuda()
    spec = api.RunSpec.from_workload(wl64, mode="variant_waves")
    with pytest.raises(RuntimeError, match="trace"):
        api.propagate(dm, spec, scales=sc64, trace_steps=8, n_trace=4)
    x0 = dm.state.clone().requires_grad_(True)
    with pytest.raises(RuntimeError, match="MT_MODE_PLAIN"):
        api.transport(x0, sc64.clone(), dm.q, spec)
