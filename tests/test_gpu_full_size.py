"""GPU parity at the benchmark sizes, in the launch forms bench.py times:
the full workloads run on the GPU and the FP64 oracle recomputes a sample
of their lanes one by one (first, last and random lanes)."""
import numpy as np
import pytest

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


def _sample(n, k, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, 1, n - 2, n - 1], rng.choice(n, k, replace=False)]))


def test_block_full_size_plain():
    """10^6 muons in the plain launch (the block workload's bench form)."""
    wl = W.make_workload("block")
    n = len(wl.muons)
    g = gpu_run(wl, mode="plain")
    idx = _sample(n, 3000, 1)
    s = compare(g, oracle_run(wl, idx), sel=idx, label="block full plain")
    print("block full plain", s)


def test_scan_full_size_variant_waves():
    """64 variants x 2^17 muons in one graph-captured variant-wave launch (the
    design scan's bench form): sampled (variant, muon) lanes of four
    variants against the oracle."""
    wl = W.make_workload("scan")
    n, v = len(wl.muons), wl.run.n_variants
    assert (n, v) == (1 << 17, 64)
    g = gpu_run(wl, mode="variant_waves", use_graph=True)
    assert g["status"].shape == (n * v,)
    for var in (0, 21, 42, 63):
        idx = _sample(n, 600, 10 + var)
        s = compare(g, oracle_run(wl, idx, variant=var), sel=var * n + idx,
                    label=f"scan full v={var}")
        print("scan full", var, s)


@pytest.mark.parametrize("mode", ["plain", "persistent"])
def test_shield_full_size(mode):
    """10^7 muons through the 40-box shield with the trilinear map."""
    wl = W.make_workload("shield")
    n = len(wl.muons)
    assert n == 10_000_000
    g = gpu_run(wl, mode=mode)
    idx = _sample(n, 1500, 2)
    s = compare(g, oracle_run(wl, idx), sel=idx, max_tie_frac=0.02, label=f"shield full {mode}",
                **map_deltas(wl))
    print("shield full", mode, s)
