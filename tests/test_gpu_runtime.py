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
    assert t["compact_every"] in (4, 8, 16, 32, 64, 128) and t["ms"] > 0
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
