"""Host checks of bench.py's bookkeeping (no GPU): the operation-class model
behind the ALU roofline, the mix-weighted peak, and the one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_operation_totals():
    """The class split of each step part adds up to its documented total."""
    totals = {k: sum(v.values()) for k, v in bench.OPS.items()}
    assert totals == {"material": 233, "vacuum": 40, "map": 30, "straight": -84,
                      "block_lookup": 43, "field_step": 120}
    assert sum(bench.SAMPLE.values()) == 113
    assert all(v >= 0 for v in bench.OPS["field_step"].values())
    assert sum(bench.PHILOX.values()) == 53
    assert all(bench.OPS["material"][c] >= v for c, v in bench.PHILOX.items())
    assert set().union(*(v.keys() for v in bench.OPS.values())) <= set(bench.CLASS_CYCLES)


def test_mix_peak_limits():
    """A pure-FP32 mix issues at twice the base rate, any other pure class at
    the base rate, and a mix lies between."""
    base = bench.VALU_BASE_LANE_OPS
    assert bench.alu_peak({"f32": 10.0}) == pytest.approx(2 * base)
    for c in ("f64", "int", "mad64", "trans"):
        assert bench.alu_peak({c: 7.0}) == pytest.approx(base)
    mix = bench._ops((1, "material"))
    assert base < bench.alu_peak(mix) < 2 * base
    # 127 FP32 ops at 2 cycles and 106 others at 4: 233 ops in 466 cycle-units
    assert bench.alu_peak(mix) == pytest.approx(233 / (127 * 2 + 106 * 4) * 4 * base)


def test_algorithmic_ops_per_workload():
    steps, lanes = 1000, 10
    blk = bench.algorithmic_ops("block", steps, lanes)
    assert sum(blk.values()) == (steps - lanes) * 233 + lanes * 40
    vw = bench.algorithmic_ops("scan", steps, lanes, "variant_waves", 64)
    assert sum(vw.values()) == pytest.approx((steps - lanes) * (233 - 53 + 53 / 64) + lanes * 40)
    vw8 = bench.algorithmic_ops("scan", steps, lanes, "variant_waves", 24)   # G = 8
    assert sum(vw8.values()) == pytest.approx((steps - lanes) * (233 - 53 + 53 / 8) + lanes * 40)
    assert [bench.share_group(v) for v in (1, 3, 8, 12, 64, 96, 128)] == [1, 1, 8, 4, 64, 32, 64]
    assert sum(bench.algorithmic_ops("shield", steps, lanes).values()) == steps * (233 + 30)
    assert sum(bench.algorithmic_ops("blocks", steps, lanes).values()) == steps * (233 + 43)
    mix = {"mat_field": 0.5, "mat_nofield": 0.25, "vac_field": 0.125, "vac_nofield": 0.125}
    sh = bench.algorithmic_ops("shield", steps, lanes, mix=mix)
    assert sum(sh.values()) == pytest.approx(steps * (0.5 * 263 + 0.25 * (233 - 84 + 30) +
                                                      0.125 * 150 + 0.125 * 70))
    bl = bench.algorithmic_ops("blocks", steps, lanes, mix=mix)
    assert sum(bl.values()) == pytest.approx(steps * (0.5 * 276 + 0.25 * (233 - 84 + 43) +
                                                      0.125 * 163 + 0.125 * 83))
    tiny = bench.algorithmic_ops("tiny", steps, lanes)
    assert sum(tiny.values()) == (steps - lanes) * (233 - 84) + lanes * 40


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_adjoint_bytes():
    """Replay-and-reverse adjoint: 51 bytes per muon-step (12-byte kick
    record read twice, 12-byte history written and read, a 48-byte
    checkpoint per 16 steps) and 112 + 8 n_mag bytes per lane."""
    assert bench.adjoint_bytes(1600, 0, 8) == 1600 * 51
    assert bench.adjoint_bytes(0, 10, 8) == 10 * (112 + 64)
    assert bench.adjoint_bytes(16, 1, 0) == 16 * 51 + 112
