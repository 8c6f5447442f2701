"""Shared helpers of the GPU parity tests: run the HIP path through the
binding, run the oracle on the same muons, and compare.

Parity bar (GPU FP32 stages with FP64 state vs the FP64 oracle):
  - muons whose oracle decision margin is below DELTA_POS (positions, m) or
    DELTA_P (relative momentum) are "tie class": a decision there can go
    either way under rounding and they are left out of the exact comparison
    (and counted);
  - for all other muons: status, step count, final volume and the per-step
    (volume, momentum bin, cell) trace agree exactly; final positions within
    1e-4 * max(|r|, 1 m) and momenta within 1e-4 * |p|.
"""
import numpy as np

import oracle

DELTA_POS = 2e-5     # m
DELTA_P = 2e-6       # relative
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
    sc = scales
    if sc is None and wl.run.scales is not None:
        sc = np.asarray(wl.run.scales, np.float64)
    return oracle.propagate(wl, np.asarray(idx, np.int64), variant=variant,
                            trace_steps=trace_steps, scales=sc)


def compare(gpu, ora, sel=None, trace_rows=None, max_tie_frac=0.01, label=""):
    """Compare GPU lanes ``sel`` (default all) with the oracle result rows.

    ``trace_rows``: number of leading compared muons whose traces both sides
    recorded.  Returns a dict of statistics."""
    if sel is None:
        sel = np.arange(len(ora.status))
    st_g = gpu["state"][:, sel]
    tie = (ora.margin_pos < DELTA_POS) | (ora.margin_p < DELTA_P)
    ok = ~tie
    n = len(sel)
    stats = {"n": n, "tie": int(tie.sum())}
    assert tie.mean() <= max_tie_frac, f"{label}: {tie.sum()} of {n} muons are tie class"
    for key, g_arr, o_arr in (("status", gpu["status"][sel], ora.status),
                              ("n_steps", gpu["n_steps"][sel], ora.n_steps),
                              ("volume", gpu["volume"][sel], ora.volume)):
        bad = np.flatnonzero(ok & (g_arr != o_arr))
        assert bad.size == 0, (f"{label}: {key} differs for {bad.size} non-tie muons, e.g. lane "
                               f"{sel[bad[0]]}: gpu {g_arr[bad[0]]} oracle {o_arr[bad[0]]}")
    valid = ok & (ora.status != oracle.ST_INVALID)
    r_o, r_g = ora.state[:3], st_g[:3]
    p_o, p_g = ora.state[3:], st_g[3:]
    dr = np.linalg.norm(r_g - r_o, axis=0)
    dp = np.linalg.norm(p_g - p_o, axis=0)
    rs = np.maximum(np.linalg.norm(r_o, axis=0), 1.0)
    ps = np.linalg.norm(p_o, axis=0)
    rel_r = np.where(valid, dr / rs, 0.0)
    rel_p = np.where(valid, dp / np.where(ps > 0, ps, 1.0), 0.0)
    stats["max_rel_r"] = float(rel_r.max()) if n else 0.0
    stats["max_rel_p"] = float(rel_p.max()) if n else 0.0
    stats["max_abs_r"] = float(np.where(valid, dr, 0).max()) if n else 0.0
    assert stats["max_rel_r"] <= REL_TOL, f"{label}: position error {stats['max_rel_r']:.3g}"
    assert stats["max_rel_p"] <= REL_TOL, f"{label}: momentum error {stats['max_rel_p']:.3g}"
    if trace_rows:
        tg = gpu["trace"][:trace_rows]
        to = ora.trace[:trace_rows]
        for j in range(trace_rows):
            if not ok[j]:
                continue
            k = int(ora.n_steps[j])
            kk = min(k, tg.shape[1])
            assert np.array_equal(tg[j, :kk], to[j, :kk]), f"{label}: trace differs, muon {j}"
    return stats
