"""Pins of the oracle's finite-difference gradients of the detector loss.

The loss is the sum over muons that leave through z_max of
sigmoid((r_ap - r)/r_scale), r being the radius at the plane z = 30 m reached
on a straight line.  Closed forms: with no field and no material the final
radius is an explicit function of the initial state; in vacuum slabs of
uniform field the path is a chain of exact circular arcs.  The oracle's
central differences must equal those of the closed forms taken with the same
step h, and the derivative with respect to a common scale of all magnets must
equal the sum of the per-magnet derivatives.
"""
import math

import numpy as np

import oracle
from paper_2512_10520_amd import workloads as W
from tests import _custom as CU

KAPPA = 0.299792458
Z_DET, R_AP, R_SC = 30.0, 1.0, 0.01


def _sig(a):
    return 1.0 / (1.0 + np.exp(-a))


def _loss_closed(xd, yd):
    return _sig((R_AP - np.sqrt(xd * xd + yd * yd)) / R_SC)


def test_fd_inputs_straight_line():
    rng = np.random.default_rng(8)
    n = 40
    x0 = rng.uniform(0.6, 1.0, n)
    y0 = rng.uniform(-0.3, 0.3, n)
    px = rng.normal(0, 0.1, n)
    py = rng.normal(0, 0.1, n)
    pz = rng.uniform(20, 80, n)
    mu = CU.muons(x0, y0, -0.0075, px, py, pz, 1)
    hist = CU.flat_histograms()
    geom = CU.geometry(np.zeros((0, 6)), np.zeros(0), world=(50.0, 50.0, 5.0))
    wl = CU.workload(hist, geom, mu, max_steps=400, p_min=0.1)
    h = 1e-3
    g, flag = oracle.fd_inputs(wl, np.arange(n), h=h, comps=(0, 1, 3, 4, 5))
    assert not flag.any()

    def closed(st):
        x, y, z, a, b, c = st
        return _loss_closed(x + (Z_DET - z) * a / c, y + (Z_DET - z) * b / c)

    st0 = mu.stacked()
    for a in (0, 1, 3, 4, 5):
        sp, sm = st0.copy(), st0.copy()
        sp[a] += h
        sm[a] -= h
        ref = (closed(sp) - closed(sm)) / (2 * h)
        assert np.allclose(g[a], ref, rtol=1e-7, atol=1e-9), a
    # d x_d / d x0 = 1: a shift of x0 moves the plane position by the same amount
    lp = oracle.detector_loss_terms
    r0 = oracle.propagate(wl)
    st = r0.state
    xd = st[0] + (Z_DET - st[2]) * st[3] / st[5]
    sh = st0.copy()
    sh[0] += 0.01
    r1 = oracle.propagate(wl, muons=sh)
    xd1 = r1.state[0] + (Z_DET - r1.state[2]) * r1.state[3] / r1.state[5]
    assert np.allclose(xd1 - xd, 0.01, atol=1e-12)
    assert lp(st, r0.status).shape == (n,)


def _arc(x, z, th, p, w, S):
    """Exact motion over arc length S at turn rate w (per metre) in the x-z
    plane, direction (-sin th, 0, cos th)."""
    if isinstance(w, complex) or np.iscomplexobj(w):
        pass
    th1 = th + w * S
    return x + (np.cos(th1) - np.cos(th)) / w, z + (np.sin(th1) - np.sin(th)) / w, th1


def test_fd_scales_two_field_slabs_closed_form():
    B0 = float(np.float32(1.7))
    hist = CU.flat_histograms()
    geom = CU.geometry([[-50, 50, -50, 50, 0.0, 2.5], [-50, 50, -50, 50, 2.5, 5.0]], [-1, -1],
                       b_box=[[0, B0, 0], [0, B0, 0]], magnet=[0, 1], n_mag=2,
                       world=(50.0, 50.0, 5.0))
    rng = np.random.default_rng(3)
    n = 12
    x0 = rng.uniform(-0.3, 0.3, n)
    p0 = rng.uniform(30.0, 120.0, n)
    q = np.where(np.arange(n) % 2 == 0, 1, -1)
    mu = CU.muons(x0, 0.0, -0.0075, 0.0, 0.0, p0, q)
    scales = np.array([[0.9, 1.1]])
    wl = CU.workload(hist, geom, mu, max_steps=400, p_min=0.1, scales=scales)
    h = 1e-3
    g, flag = oracle.fd_scales(wl, np.arange(n), h=h)
    assert not flag.any()
    tr = oracle.propagate(wl, trace_steps=400)

    def closed(s, j):
        vols = tr.trace[j, : tr.n_steps[j], 0]
        x, z, th = x0[j], -0.0075, 0.0
        for v in vols:                       # one exact arc per step, field of its box
            if v < 0:
                x, z = x - 0.02 * np.sin(th), z + 0.02 * np.cos(th)
            else:
                w = KAPPA * q[j] * s[v] * B0 / p0[j]
                x, z, th = _arc(x, z, th, p0[j], w, 0.02)
        xd = x + (Z_DET - z) * (-np.tan(th))
        return _loss_closed(xd, 0.0)

    for m in range(2):
        ref = 0.0
        for j in range(n):
            sp, sm = scales[0].copy(), scales[0].copy()
            sp[m] += h
            sm[m] -= h
            ref += (closed(sp, j) - closed(sm, j)) / (2 * h)
        assert abs(g[m] - ref) <= 1e-7 * max(1.0, abs(ref)), (m, g[m], ref)
    # the closed form has a non-trivial gradient for both magnets
    assert np.all(np.abs(g) > 1e-3)


def test_fd_common_scale_equals_sum_of_magnet_derivatives():
    wl = W.make_workload("diff", n_muons=300, n_fill=20_000)
    idx = np.arange(300)
    h = 1e-3
    g, flag = oracle.fd_scales(wl, idx, h=h)
    base = np.asarray(wl.run.scales, np.float64)
    rp = oracle.propagate(wl, idx, scales=base * (1 + h), trace_steps=wl.run.max_steps)
    rm = oracle.propagate(wl, idx, scales=base * (1 - h), trace_steps=wl.run.max_steps)
    flag2 = flag | (rp.trace != rm.trace).any(axis=(1, 2)) | (rp.n_steps != rm.n_steps)
    lp = oracle.detector_loss_terms(rp.state, rp.status)
    lm = oracle.detector_loss_terms(rm.state, rm.status)
    total = np.sum(np.where(flag2, 0.0, (lp - lm) / (2 * h)))
    # recompute the per-magnet sum over the same kept muons
    g2, _ = oracle.fd_scales(wl, idx[~flag2], h=h)
    assert flag2.mean() < 0.2
    assert abs(total - g2.sum()) <= 2e-3 * max(1.0, abs(total)), (total, g2.sum())


def _fnv1a(trace_rows):
    """64-bit FNV-1a over the little-endian bytes of the (vol, bin, cell) rows."""
    h = 0xCBF29CE484222325
    for b in np.ascontiguousarray(trace_rows, dtype="<i4").tobytes():
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_trace_digest_is_the_hash_of_the_whole_trace():
    """The finite-difference helpers flag a muon when its decision path
    differs between the +h and -h runs, comparing 64-bit digests of the
    paths instead of storing them.  The digest must be the FNV-1a hash of
    every step's (volume, bin, cell), and muons with different paths must get
    different digests (here: every muon of a short block run differs)."""
    wl = W.make_workload("block", n_muons=60, n_fill=20_000)
    r = oracle.propagate(wl, np.arange(60), trace_steps=wl.run.max_steps, digest=True)
    for j in range(60):
        k = int(r.n_steps[j])
        assert int(r.digest[j]) == _fnv1a(r.trace[j, :k]), j
    assert len(set(r.digest.tolist())) == 60
    # same path, same digest, whatever else differs: scaling all magnet fields
    # by 1 + 1e-12 leaves the (vol, bin, cell) path of nearly every muon as is
    wl2 = W.make_workload("diff", n_muons=40, n_fill=20_000)
    a = oracle.propagate(wl2, np.arange(40), trace_steps=wl2.run.max_steps, digest=True)
    b = oracle.propagate(wl2, np.arange(40), trace_steps=wl2.run.max_steps, digest=True,
                         scales=np.full((1, wl2.geom.n_mag), 1.0 + 1e-12))
    same = (a.trace == b.trace).all(axis=(1, 2))
    assert same.sum() >= 35
    assert np.array_equal(a.digest[same], b.digest[same])
    assert not np.array_equal(a.state, b.state)
