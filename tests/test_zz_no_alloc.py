"""GPU: mt_propagate_noalloc, the entry point for callers that cannot
allocate device memory, gives mt_propagate's results bit for bit.

Its workspace (the persistent form's work counter, the tally partial sums)
is a fixed device array shared by every call on the device, so the test
makes two calls in a row, the second with a smaller input, in each launch
form that uses the workspace (persistent with tallies) and in the plain
form, and checks both against mt_propagate on the same inputs.  It also
checks the documented limit: a tally whose partial sums do not fit is
rejected with MT_ERR_LIMIT before any launch."""
import numpy as np
import pytest

from paper_2512_10520_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("state", "status", "n_steps", "volume", "tally")
TALLY = {"z_det": 30.0, "r_ap": 1.0, "r_scale": 0.01}


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    return t


def _run(torch, api, wl, n, mode, noalloc, n_variants):
    dm = api.DeviceMuons.from_host(wl.muons.take(np.arange(n)))
    spec = api.RunSpec.from_workload(wl, mode=mode)
    spec.n_variants = n_variants
    sc = torch.from_numpy(np.ascontiguousarray(wl.run.scales[:n_variants], np.float32)).cuda()
    out = api.alloc_result(spec, n, "cuda", tally=True)
    api.propagate(dm, spec, scales=sc, tally=TALLY, out=out, noalloc=noalloc)
    torch.cuda.synchronize()
    return {k: getattr(out, k).cpu().numpy() for k in KEYS}


@pytest.mark.parametrize("mode", ["persistent", "plain"])
def test_noalloc_equals_propagate_twice(torch, mode):
    from paper_2512_10520_amd import api
    wl = W.make_workload("scan", n_muons=30_000, n_variants=8, n_fill=200_000)
    api.load_workload(wl)
    for n in (30_000, 7_777):               # the second call is smaller
        ref = _run(torch, api, wl, n, mode, False, 8)
        got = _run(torch, api, wl, n, mode, True, 8)
        for k in KEYS:
            assert np.array_equal(ref[k], got[k]), (mode, n, k)
        assert ref["tally"][:, 0].sum() > 0


def test_noalloc_rejects_what_does_not_fit(torch):
    """Tally partial sums beyond the fixed workspace (10 partial blocks x 4400
    variants x 24 B > 1 MiB) and graph capture are rejected by the host check
    that precedes every launch, so no kernel runs and the small buffers given
    here are never touched."""
    import ctypes as C
    from paper_2512_10520_amd import _lib, api
    wl = W.make_workload("scan", n_muons=4096, n_variants=8, n_fill=20_000)
    api.load_workload(wl)
    L = _lib.load()
    n, nv = 40_960, 4_400
    dm = api.DeviceMuons.from_host(wl.muons)
    out = api.alloc_result(api.RunSpec.from_workload(wl), len(dm), "cuda", tally=True)
    sc = torch.ones((1, wl.geom.n_mag), dtype=torch.float32, device="cuda")
    spec = api.RunSpec.from_workload(wl, mode="persistent")
    spec.n_variants = nv
    p = api._params(spec, sc, tally=out.tally, **TALLY)
    res = _lib.MtResult(out.status.data_ptr(), out.n_steps.data_ptr(), out.volume.data_ptr())
    o = _lib.MtMuons(*[out.state[a].data_ptr() for a in range(6)], None)
    i = dm.c_struct()
    rc = L.mt_propagate_noalloc(C.byref(p), n, C.byref(i), C.byref(o), C.byref(res), None)
    assert rc == -7 and "MT_NOALLOC_SCRATCH_BYTES" in api.last_error()
    spec.n_variants = 1
    spec.use_graph = True
    p = api._params(spec, sc)
    rc = L.mt_propagate_noalloc(C.byref(p), len(dm), C.byref(i), C.byref(o), C.byref(res), None)
    assert rc == -1 and "use_graph" in api.last_error()
    torch.cuda.synchronize()
