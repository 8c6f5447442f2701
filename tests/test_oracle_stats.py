"""Statistical pins of the oracle's sampler and kick.

One transport step from p = (0, 0, P) with no field leaves
p' = P (tau cos phi, tau sin phi, 1 - f), so (f, tau, phi) can be read back
from the final state and compared with the source histogram (chi-square on
the 2D cells and on both marginals, uniformity inside the cell, isotropic
azimuth).  Over many steps the log of the momentum magnitude is a sum of
i.i.d. terms 0.5 ln((1 - f)^2 + tau^2) whose mean and variance follow from
integrals over the histogram cells.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2512_10520_amd import workloads as W
from tests import _custom as CU


SAMPLERS = pytest.mark.parametrize("sampler", [0, 1], ids=["cdf", "alias"])


def _one_step(hist, n, P=100.0, sampler=0):
    geom = CU.geometry([[-10, 10, -10, 10, 0, 100]], [0])
    mu = CU.muons(np.zeros(n), 0.0, 0.01, 0.0, 0.0, P, 1)
    wl = CU.workload(hist, geom, mu, max_steps=1, p_min=0.1, sampler=sampler)
    res = oracle.propagate(wl)
    assert np.all(res.n_steps == 1)
    px, py, pz = res.state[3:]
    f = 1.0 - pz / P
    tau = np.hypot(px, py) / P
    phi = np.mod(np.arctan2(py, px), 2 * math.pi)
    return f, tau, phi


def _cells(hist, f, tau):
    """Cell indices and position inside the cell (in the axis' own units:
    log10 on a logarithmic axis) of recovered (f, tau) values."""
    def axis(v, lo, hi, n, lg):
        if lg:
            v, lo, hi = np.log10(v), math.log10(lo), math.log10(hi)
        return (v - lo) / ((hi - lo) / n) + 1e-9
    la = getattr(hist, "log_axes", (False, False))
    ul = axis(f, hist.loss_lo, hist.loss_hi, hist.n_loss, la[0])
    us = axis(tau, hist.scat_lo, hist.scat_hi, hist.n_scat, la[1])
    il, is_ = np.floor(ul).astype(np.int64), np.floor(us).astype(np.int64)
    return il, is_, ul - il, us - is_


def _chi2_p(obs, expected):
    keep = expected >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(expected[keep], expected[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    return stats.chisquare(o, e * o.sum() / e.sum()).pvalue


@SAMPLERS
def test_sampled_cells_and_marginals_match_histogram(sampler):
    hist = CU.flat_histograms(n_pbin=4, n_loss=8, n_scat=8, seed=21)
    n = 1_000_000
    f, tau, phi = _one_step(hist, n, sampler=sampler)
    il, is_, fl, fs = _cells(hist, f, tau)
    counts = hist.counts[0, 0].astype(np.float64)
    assert il.min() >= 0 and il.max() < 8 and is_.min() >= 0 and is_.max() < 8
    obs = np.bincount(il * 8 + is_, minlength=64).astype(np.float64)
    assert np.all(obs[counts.ravel() == 0] == 0)                 # empty cells never drawn
    exp = n * counts.ravel() / counts.sum()
    assert _chi2_p(obs, exp) > 1e-4
    assert _chi2_p(obs.reshape(8, 8).sum(1), exp.reshape(8, 8).sum(1)) > 1e-4
    assert _chi2_p(obs.reshape(8, 8).sum(0), exp.reshape(8, 8).sum(0)) > 1e-4
    # jitter: uniform inside the drawn cell on both axes; azimuth isotropic
    assert stats.kstest(fl[:200_000], "uniform").pvalue > 1e-4
    assert stats.kstest(fs[:200_000], "uniform").pvalue > 1e-4
    assert stats.kstest(phi[:200_000] / (2 * math.pi), "uniform").pvalue > 1e-4
    # the two jitters and the azimuth are independent of each other
    assert abs(np.corrcoef(fl, fs)[0, 1]) < 5 / math.sqrt(n)
    assert abs(np.corrcoef(fl, phi)[0, 1]) < 5 / math.sqrt(n)


@SAMPLERS
def test_sampled_cells_realistic_histogram(sampler):
    wl = W.make_workload("tiny", n_muons=1)
    hist = wl.hist
    n = 500_000
    f, tau, _ = _one_step(hist, n, P=100.0, sampler=sampler)   # 100 GeV: momentum bin 24
    il, is_, _, _ = _cells(hist, f, tau)
    counts = hist.counts[0, 24].astype(np.float64).ravel()
    obs = np.bincount(il * hist.n_scat + is_, minlength=counts.size).astype(np.float64)
    assert np.all(obs[counts == 0] == 0)
    assert _chi2_p(obs, n * counts / counts.sum()) > 1e-4


def _cell_moments(hist):
    """E[g] and E[g^2] of g = 0.5 ln((1-f)^2 + tau^2) for the piecewise-uniform
    density of the histogram, by 24-point Gauss-Legendre on every cell."""
    x, w = np.polynomial.legendre.leggauss(24)
    wl_ = (hist.loss_hi - hist.loss_lo) / hist.n_loss
    ws_ = (hist.scat_hi - hist.scat_lo) / hist.n_scat
    c = hist.counts[0, 0].astype(np.float64)
    prob = c / c.sum()
    m1 = m2 = 0.0
    for a in range(hist.n_loss):
        fa = hist.loss_lo + (a + 0.5 * (x + 1)) * wl_
        for b in range(hist.n_scat):
            if prob[a, b] == 0:
                continue
            tb = hist.scat_lo + (b + 0.5 * (x + 1)) * ws_
            F, T = np.meshgrid(fa, tb, indexing="ij")
            g = 0.5 * np.log((1 - F) ** 2 + T ** 2)
            ww = np.outer(w, w) / 4
            m1 += prob[a, b] * np.sum(ww * g)
            m2 += prob[a, b] * np.sum(ww * g * g)
    return m1, m2


@SAMPLERS
def test_log_momentum_moments_over_many_steps(sampler):
    hist = CU.flat_histograms(n_pbin=4, n_loss=8, n_scat=8, seed=9, p_lo=1.0, p_hi=1000.0)
    n, N = 100_000, 50
    geom = CU.geometry([[-10, 10, -10, 10, 0, 100]], [0])
    mu = CU.muons(np.zeros(n), 0.0, 0.01, 0.0, 0.0, 100.0, 1)
    res = oracle.propagate(CU.workload(hist, geom, mu, max_steps=N, p_min=0.1,
                                       sampler=sampler))
    assert np.all(res.n_steps == N) and np.all(res.status == oracle.ST_STEPS)
    s = np.log(np.linalg.norm(res.state[3:], axis=0) / 100.0)
    m1, m2 = _cell_moments(hist)
    var_g = m2 - m1 * m1
    se = math.sqrt(N * var_g / n)
    assert abs(s.mean() - N * m1) < 5 * se, (s.mean(), N * m1, se)
    # steps draw independent words: the variance of the sum is N Var[g]
    assert abs(s.var() / (N * var_g) - 1) < 0.03


@SAMPLERS
def test_log_axes_cells_and_in_cell_uniformity(sampler):
    """Histograms binned in log10 of f and tau (Section "Building
    histograms"): the drawn cells follow the counts and the jitter is uniform
    in log10 inside the cell (so f itself is not uniform in the cell)."""
    rng = np.random.default_rng(31)
    counts = rng.integers(0, 60, size=(8, 8)).astype(np.uint32)
    counts[0, 3] = 0
    hist = CU.flat_histograms(counts=counts, loss=(1e-4, 0.1), scat=(1e-5, 1e-2))
    hist.log_axes = (True, True)
    n = 600_000
    f, tau, _ = _one_step(hist, n, sampler=sampler)
    il, is_, fl, fs = _cells(hist, f, tau)
    assert il.min() >= 0 and il.max() < 8 and is_.min() >= 0 and is_.max() < 8
    obs = np.bincount(il * 8 + is_, minlength=64).astype(np.float64)
    exp = n * counts.ravel() / counts.sum()
    assert np.all(obs[counts.ravel() == 0] == 0)
    assert _chi2_p(obs, exp) > 1e-4
    assert stats.kstest(fl[:200_000], "uniform").pvalue > 1e-4
    assert stats.kstest(fs[:200_000], "uniform").pvalue > 1e-4
    # in linear units the position inside a loss cell is not uniform
    lo = 10 ** (math.log10(1e-4) + il * (3.0 / 8))
    hi = 10 ** (math.log10(1e-4) + (il + 1) * (3.0 / 8))
    assert stats.kstest(((f - lo) / (hi - lo))[:200_000], "uniform").pvalue < 1e-6
