"""Shared helpers of the GPU parity tests: run the HIP path through the
binding, run the oracle on the same muons, and compare.

Parity bar (GPU FP32 stages with FP64 state vs the FP64 oracle):
  - status, step count, final volume and the per-step (volume, momentum bin,
    cell) trace agree exactly, final positions within 1e-4 * max(|r|, 1 m)
    and momenta within 1e-4 * |p|;
  - except for "tie" muons: a muon may part ways with the oracle only at a
    decision whose oracle margin is below DELTA_POS (distance to a face or
    threshold, m) or DELTA_P (relative distance of |p| to a bin edge or to
    p_min).  Such a decision can go either way under rounding; these muons
    are counted and their number is bounded per test.
DELTA_POS and DELTA_P are at least 10x the largest GPU-oracle deviation of
the agreeing muons observed in these tests.  With a field map the state
deviations at the steps where decisions are taken are larger (the map's
interpolation weights are formed from the FP32-stepped state, and the long
shield paths hold low-momentum muons that curl in strong fields), so map
workloads use the deltas of MAP_DELTAS for their field options, each at
least 10x the largest deviation measured at decision time for that option
(tests/test_gpu_parity.py, test_shield_decision_time_deviation; largest
position / relative momentum deviations over 46 000 (muon, step) pairs:
trilinear 1.3e-5 m / 5.9e-6, alias sampler 4.2e-5 m / 6.6e-6, nearest node
9.1e-6 m / 4.1e-7, field at every stage 8.6e-6 m / 6.2e-6, nearest node
and every stage 1.0e-4 m / 3.1e-5).
"""
import numpy as np

import oracle

DELTA_POS = 1e-5     # m
DELTA_P = 1e-6       # relative
# (interp, stage_field, sampler) of a workload with a field map -> (m, relative)
MAP_DELTAS = {(0, 0, 0): (2e-4, 1e-4), (0, 0, 1): (5e-4, 1e-4), (1, 0, 0): (1e-4, 1e-5),
              (0, 1, 0): (1e-4, 1e-4), (1, 1, 0): (1.2e-3, 4e-4)}


def map_deltas(wl):
    """Tie deltas (compare() keywords) of a workload with a field map."""
    r = wl.run
    key = (int(getattr(r, "interp", 0)), int(getattr(r, "stage_field", 0)),
           int(getattr(r, "sampler", 0)))
    if key not in MAP_DELTAS:             # e.g. alias with nearest node: the widest
        key = (1, 1, 0)
    dpos, dp = MAP_DELTAS[key]
    return {"delta_pos": dpos, "delta_p": dp}
REL_TOL = 1e-4


def gpu_run(wl, n=None, mode="plain", trace_steps=0, n_trace=0, scales=None, block=0,
            compact_every=0, use_graph=False, n_variants=None, tally=None):
    import torch
    from paper_2512_10520_amd import api
    api.load_workload(wl)
    mu = wl.muons if n is None else wl.muons.take(np.arange(n))
    dm = api.DeviceMuons.from_host(mu)
    spec = api.RunSpec.from_workload(wl, mode=mode, block=block, compact_every=compact_every,
                                     use_graph=use_graph)
    if n_variants is not None:
        spec.n_variants = n_variants
    sc = None
    if scales is not None:
        sc = torch.from_numpy(np.ascontiguousarray(scales, np.float32)).cuda()
    elif wl.run.scales is not None:
        sc = torch.from_numpy(np.ascontiguousarray(wl.run.scales[:spec.n_variants],
                                                   np.float32)).cuda()
    res = api.propagate(dm, spec, scales=sc, trace_steps=trace_steps, n_trace=n_trace,
                        tally=tally)
    torch.cuda.synchronize()
    out = {"state": res.state.cpu().numpy(), "status": res.status.cpu().numpy(),
           "n_steps": res.n_steps.cpu().numpy(), "volume": res.volume.cpu().numpy()}
    if res.trace is not None:
        out["trace"] = res.trace.cpu().numpy()
    if res.tally is not None:
        out["tally"] = res.tally.cpu().numpy()
    return out


def oracle_run(wl, idx, variant=None, trace_steps=0, scales=None):
    """Oracle on muons idx (Philox indices), with per-step traces and margins
    when trace_steps > 0."""
    sc = scales
    if sc is None and wl.run.scales is not None:
        sc = np.asarray(wl.run.scales, np.float64)
    return oracle.propagate(wl, np.asarray(idx, np.int64), variant=variant,
                            trace_steps=trace_steps, scales=sc)


def _differs(gpu, ora, sel, i):
    """Does lane sel[i] differ from oracle row i beyond the parity bar?"""
    g = sel[i]
    if (gpu["status"][g] != ora.status[i] or gpu["n_steps"][g] != ora.n_steps[i] or
            gpu["volume"][g] != ora.volume[i]):
        return True
    if ora.status[i] == oracle.ST_INVALID:
        return False
    r_o, p_o = ora.state[:3, i], ora.state[3:, i]
    r_g, p_g = gpu["state"][:3, g], gpu["state"][3:, g]
    if np.linalg.norm(r_g - r_o) > REL_TOL * max(np.linalg.norm(r_o), 1.0):
        return True
    return np.linalg.norm(p_g - p_o) > REL_TOL * np.linalg.norm(p_o)


def compare(gpu, ora, sel=None, trace_rows=0, max_tie_frac=0.01, label="", delta_pos=DELTA_POS,
            delta_p=DELTA_P):
    """Compare GPU lanes ``sel`` (default 0..n-1) with the oracle rows.

    A muon may differ only through a boundary tie.  For muons with a trace on
    both sides (the first ``trace_rows`` rows, oracle run with per-step
    margins) the first step where the (volume, bin, cell) traces, the step
    count, the status or the final volume part ways must be a step whose
    oracle decision margin is below DELTA_POS / DELTA_P.  For the other muons
    the minimum margin over the whole trajectory must be below them.
    Everything else must agree: discrete outputs exactly, states within
    REL_TOL.  Returns statistics (including the largest position / momentum
    deviations of the agreeing muons, used to calibrate the deltas)."""
    n = len(ora.status)
    sel = np.arange(n) if sel is None else np.asarray(sel)
    agree = np.ones(n, bool)
    tie = np.zeros(n, bool)
    for i in range(n):
        g = sel[i]
        diverge_k = None
        if i < trace_rows:
            T = gpu["trace"].shape[1]
            m = int(min(gpu["n_steps"][g], ora.n_steps[i], T))
            d = np.flatnonzero((gpu["trace"][g, :m] != ora.trace[i, :m]).any(axis=1))
            if d.size:
                diverge_k = int(d[0])
            elif _differs(gpu, ora, sel, i):
                diverge_k = m
        elif _differs(gpu, ora, sel, i):
            diverge_k = -1
        if diverge_k is None:
            continue
        agree[i] = False
        if diverge_k >= 0 and ora.step_margin is not None and diverge_k < ora.step_margin.shape[1] \
                and not (diverge_k == gpu["trace"].shape[1] and ora.n_steps[i] > diverge_k):
            mpos, mp = ora.step_margin[i, diverge_k]
        else:
            mpos, mp = ora.margin_pos[i], ora.margin_p[i]
        if mpos < delta_pos or mp < delta_p:
            tie[i] = True
        else:
            raise AssertionError(
                f"{label}: lane {g} differs from the oracle with no boundary tie "
                f"(first divergence at step {diverge_k}, margins pos {mpos:.3g} m, p {mp:.3g}): "
                f"gpu status/steps/vol {gpu['status'][g]}/{gpu['n_steps'][g]}/{gpu['volume'][g]}, "
                f"oracle {ora.status[i]}/{ora.n_steps[i]}/{ora.volume[i]}")
    valid = agree & (ora.status != oracle.ST_INVALID)
    st_g = gpu["state"][:, sel]
    dr = np.linalg.norm(st_g[:3] - ora.state[:3], axis=0)
    dp = np.linalg.norm(st_g[3:] - ora.state[3:], axis=0)
    ps = np.linalg.norm(ora.state[3:], axis=0)
    rel_dp = np.where(valid, dp / np.where(ps > 0, ps, 1), 0)
    stats = {"n": n, "tie": int(tie.sum()),
             "max_abs_dr": float(np.where(valid, dr, 0).max()) if n else 0.0,
             "max_rel_dp": float(rel_dp.max()) if n else 0.0}
    if n:
        w = int(np.argmax(rel_dp))
        stats["worst"] = {"status": int(ora.status[w]), "n_steps": int(ora.n_steps[w]),
                          "p_final": float(ps[w])}
    assert tie.mean() <= max_tie_frac if n else True, f"{label}: {tie.sum()} of {n} muons diverged"
    return stats
