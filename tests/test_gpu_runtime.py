"""Runtime behaviour of the library on the GPU: the autotuner's choice is
valid, remembered and gives the plain launch's bits; release and reload
between geometry kinds; a sequence of loads keeps results reproducible."""
import numpy as np
import pytest

from paper_2512_10520_amd import workloads as W
from tests._parity import gpu_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2512_10520_amd import _lib
    _lib.load()


def test_autotune_choice_is_valid_and_used():
    import torch
    from paper_2512_10520_amd import api
    wl = W.make_workload("block", n_muons=30_000, n_fill=200_000)
    api.load_workload(wl)
    dm = api.DeviceMuons.from_host(wl.muons)
    spec = api.RunSpec.from_workload(wl, mode="persistent")
    t = api.autotune(dm, spec)
    assert t["block"] in (64, 128, 256, 512)
    assert t["compact_every"] in (32, 64, 128, 256, 512, 1 << 30) and t["ms"] > 0
    # a later call with block = 0 and compact_every = 0 uses the remembered
    # choice; every choice gives the plain launch's bits
    tuned = api.propagate(dm, spec)
    plain = api.propagate(dm, api.RunSpec.from_workload(wl, mode="plain"))
    torch.cuda.synchronize()
    for k in ("state", "status", "n_steps", "volume"):
        assert torch.equal(getattr(tuned, k), getattr(plain, k)), k


def test_release_and_reload_between_geometry_kinds():
    from paper_2512_10520_amd import api
    a = W.make_workload("blocks", n_muons=2000, n_fill=100_000)
    b = W.make_workload("shield", n_muons=2000, n_fill=100_000)
    ra = gpu_run(a)
    rb = gpu_run(b)
    api.release()
    with pytest.raises(RuntimeError, match="loaded"):
        api.propagate(api.DeviceMuons.from_host(a.muons), api.RunSpec.from_workload(a))
    ra2 = gpu_run(a)
    rb2 = gpu_run(b)
    for k in ra:
        assert np.array_equal(ra[k], ra2[k]), k
        assert np.array_equal(rb[k], rb2[k]), k


def test_graph_replay_after_workspace_grows():
    """A graph captured with a small tally holds the address of the library's
    tally partials.  A later call needing a larger partial buffer (a tally
    over more muons, then a backward pass with scale gradients) reallocates
    it, which drops the cached graphs; replaying the first call then
    captures again and gives the eager tally."""
    import torch
    from paper_2512_10520_amd import api
    t = {"z_det": 30.0, "r_ap": 1.0, "r_scale": 0.01}
    wl = W.make_workload("scan", n_muons=200_000, n_variants=3, n_fill=200_000)
    api.load_workload(wl)
    sc = torch.from_numpy(np.ascontiguousarray(wl.run.scales, np.float32)).cuda()
    small = api.DeviceMuons.from_host(wl.muons.take(np.arange(1000)))
    big = api.DeviceMuons.from_host(wl.muons)
    spec_g = api.RunSpec.from_workload(wl, mode="persistent", use_graph=True)
    spec_e = api.RunSpec.from_workload(wl, mode="persistent")
    eager = api.propagate(small, spec_e, scales=sc, tally=t)
    torch.cuda.synchronize()
    ref = eager.tally.cpu().numpy()
    out = api.alloc_result(spec_g, len(small), "cuda", tally=True)
    api.propagate(small, spec_g, scales=sc, tally=t, out=out)          # capture
    torch.cuda.synchronize()
    assert np.array_equal(out.tally.cpu().numpy(), ref)
    api.propagate(big, spec_e, scales=sc, tally=t)                      # partials grow
    spec_d = api.RunSpec.from_workload(wl)
    fwd = api.propagate(big, spec_d, scales=sc, ckpt=True)
    g_out = torch.ones((6, 3 * len(big)), dtype=torch.float64, device="cuda")
    api.propagate_backward(big, spec_d, fwd, g_out, scales=sc, n_mag=8)  # and again
    torch.cuda.synchronize()
    for rep in range(3):
        out.tally.fill_(-1.0)
        api.propagate(small, spec_g, scales=sc, tally=t, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.tally.cpu().numpy(), ref), rep
