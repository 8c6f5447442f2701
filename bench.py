"""Benchmark: muon-steps/s of the HIP transport on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config shield]
                    [--no-cpu] [--no-extra]

A step is one transport of the whole synthetic batch (all muons to their
break condition) with every table already resident in HBM.  The default
workload is the realistic-shaped shield: 40 boxes (magnet yokes, air cores,
concrete walls) in 8 stations over 30 m, 3 materials x 95 log momentum bins
(0.18-400 GeV) x 100 x 100 histogram cells, a 100 x 100 x 300 float32 field
map interpolated trilinearly, 10^7 power-law muons with uneven path lengths;
the reported form is the faster of the plain and the persistent launch.
The same default run adds, as extra keys, the magnetised block (10^6
muons), the batched design scan (64 field variants x 2^17 muons) and the
differentiable design step (forward with checkpoints + adjoint, 10^6
muons).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "muon-steps/sec on 1 MI355X vs CPU FP64 oracle; fwd+adjoint time per design step"

# ALU roofline.  A SIMD issues one 64-lane VALU instruction per 4 cycles at
# the base 16-lane rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13
# lane-operations/s, which is MI355X's published FP64 vector peak (78.6
# TFLOP/s counting an FMA as two).  FP32 instructions issue at twice that
# (157.3 TFLOP/s): 2 cycles per 64-lane instruction.  The peak of a step is
# therefore that of its mix: with n_c operations of class c per step and
# cost_c cycles per 64-lane instruction of the class, a SIMD completes
# 64 / sum(n_c cost_c) steps per cycle.  Integer operations, the 32x32->64
# products and the transcendentals (rsq, sin, cos) are charged the base rate
# (no published figure; optimistic for the 64-bit products).
CLOCK_HZ, SIMDS = 2.4e9, 256 * 4
CLASS_CYCLES = {"f32": 2, "f64": 4, "int": 4, "mad64": 4, "trans": 4}
VALU_BASE_LANE_OPS = SIMDS * 16 * CLOCK_HZ

# Algorithmic operations of one muon step, counted from the method at the
# granularity of single hardware operations and split by class.  A material
# step (233): break test 8 (7 FP64 compares, step cap), box lookup 6 (cached
# box: 4 FP64 compares), momentum bin 2 (FP64), Philox4x32-10 53 (18
# 32x32->64 products + 35 xors once the muon-constant part of rounds 1-2 is
# hoisted), inverse CDF 7 and cell split 3 (integer), jitter + azimuth 18
# (FP32, sin and cos), kick + rotation 30 (FP32, one rsq, the FP64 update of
# p and its conversions), field 1, RK4 103 (FP32 stages with 4 rsq, FP64
# accumulation and conversions), loop 2.  A vacuum step in zero field is 40.
# The field map adds 30 (FP64 cell coordinates and index, and 15 FP32 for the
# interpolation: a lower bound, the cell polynomial takes 21 FMAs);
# zero-field material steps replace the RK4 by the straight-line update
# (-84).  A convex-block lookup replaces the box lookup by one candidate's
# sign test (grid cell, slice and edge products in FP64: +43).  In the
# variant-wave form G lanes holding variants of one muon share one Philox
# block per step, so a lane's share of its 53 operations is 53 / G.
OPS = {
    "material": {"f32": 127, "f64": 31, "int": 50, "mad64": 18, "trans": 7},
    "vacuum": {"f32": 12, "f64": 17, "int": 9, "trans": 2},
    "map": {"f32": 15, "f64": 9, "int": 6},
    "straight": {"f32": -80, "trans": -4},
    "block_lookup": {"f64": 40, "int": 3},
}
PHILOX = {"mad64": 18, "int": 35}        # the Philox part of a material step
# The part of a material step that only a material step does (momentum bin,
# Philox, cell draw and split, jitter and azimuth, kick and rotation: 113):
# a step outside every material but inside a field does the rest (120).
SAMPLE = {"f32": 30, "f64": 14, "int": 48, "mad64": 18, "trans": 3}
OPS["field_step"] = {c: OPS["material"].get(c, 0) - SAMPLE.get(c, 0) for c in CLASS_CYCLES}


def share_group(n_variants):
    """Lanes sharing a random stream in the variant-wave form: the largest
    power of two dividing the variant count, at most 64."""
    g = 1
    while g < 64 and n_variants % (2 * g) == 0:
        g *= 2
    return g


def _ops(*parts):
    """Sum of operation-class vectors, each given as (count, OPS key)."""
    out = {c: 0.0 for c in CLASS_CYCLES}
    for count, key in parts:
        for c, v in OPS[key].items():
            out[c] += count * v
    return out


def alu_peak(ops):
    """Lane-operations/s the SIMDs can issue for this operation mix."""
    total = sum(ops.values())
    cycles = sum(v * CLASS_CYCLES[c] for c, v in ops.items())
    return total / cycles * SIMDS * CLOCK_HZ * 64


WORKLOADS = {
    "tiny": "tiny: 1 iron box 1 m, no field, 32x64x64 histograms, 10^4 muons at 100 GeV",
    "block": "block: 5 m iron box, uniform 1.7 T, 95x100x100 histograms, 10^6 power-law muons",
    "shield": "shield: 40 boxes, 3 materials, 100x100x300 trilinear field map, 10^7 muons",
    "scan": "scan: 8 iron slabs, 64 field-scale variants x 2^17 muons, one graph launch",
    "blocks": "blocks: 40 convex blocks (tapered yokes and core), 3 materials, 10^6 muons",
    "logbins": "logbins: block with log10-binned histogram axes (the paper's parameterisation)",
}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="shield", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="auto",
                    choices=["auto", "plain", "persistent", "variant_waves"],
                    help="auto: time every form the workload admits and report the fastest "
                         "(variant_waves: workloads with several field variants)")
    ap.add_argument("--block", type=int, default=0,
                    help="threads per block of the timed form (0: autotuned / default)")
    ap.add_argument("--compact", type=int, default=0,
                    help="persistent form: steps per pass (0: autotuned); with --block and a "
                         "fixed --mode the autotuner is skipped (for profiling runs)")
    ap.add_argument("--design-only", action="store_true",
                    help="time only the differentiable design step (forward with checkpoints "
                         "and adjoint, 10^6 muons) and print it")
    ap.add_argument("--sampler", default="cdf", choices=["cdf", "alias"],
                    help="histogram-cell sampler of the timed pass (the other one is timed "
                         "beside it on the block workload)")
    ap.add_argument("--interp", default="trilinear", choices=["trilinear", "nearest"],
                    help="field map lookup (workloads with a map)")
    ap.add_argument("--stage-field", action="store_true",
                    help="evaluate the field at every RK4 stage position")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="shield: skip the block, design-scan and design-step keys")
    ap.add_argument("--cpu-muons", type=int, default=0,
                    help="muons of the oracle sample (0: about 10 s of host time)")
    ap.add_argument("--gather-sweep", action="store_true",
                    help="only measure random-gather rates over a range of table sizes")
    ap.add_argument("--alu-sweep", action="store_true",
                    help="measure SIMD cycles per wave-level VALU instruction for five "
                         "instruction kinds (libmt_gbench.so) and exit")
    ap.add_argument("--no-other", action="store_true",
                    help="skip timing the other sampler beside the timed pass")
    ap.add_argument("--no-gather", action="store_true",
                    help="skip the gather-ceiling microbenchmark")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM byte counters)")
    return ap.parse_args()


def copy_calibration(torch, nbytes=1 << 30, reps=4):
    """A plain device-to-device copy of known size: FETCH_SIZE / WRITE_SIZE of
    this kernel per dispatch give the counters' scale (bytes read and written
    are nbytes each)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def _time_launches(fn, k, torch):
    """Run fn k times; return (wall seconds, mean per-launch ms from HIP events
    recorded on the launch stream)."""
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(k)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(s)
        fn()
        b.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    return wall, ev_ms


def main():
    args = _parse()
    if args.gpus != 1:
        sys.exit(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the transport "
                 "shards by muon index across GPUs, but this build runs and reports N=1.")
    import torch

    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.gather_sweep:
        rates = {f"{w}B@{b / 2 ** 20:.1f}MiB": gather_rate(torch, b, w)
                 for w, b in ((4, 1 << 19), (4, 3774874), (4, 10 << 20), (4, 11429478),
                              (16, 48023552), (16, 392 << 20))}
        print(json.dumps({"gather_loads_per_s": rates}), flush=True)
        return

    if args.alu_sweep:
        print(json.dumps({"simd_cycles_per_wave_instruction": alu_rates(torch)}), flush=True)
        return

    from paper_2512_10520_amd import api
    from paper_2512_10520_amd import workloads as W

    torch.cuda.set_device(0)
    if args.design_only:
        print(json.dumps({"design_step": design_step(api, W, torch)}), flush=True)
        return
    m = measure(api, W, torch, args.config, args.mode, args.sampler, args.interp,
                args.stage_field, args.steps, args.warmup, other_sampler=not args.no_other,
                block=args.block, compact=args.compact)
    line = {"metric": METRIC, "value": m["value"], "unit": "muon-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": m["config"], "roofline": m["roofline"]}
    for k in ("other_sampler", "per_variant_plain_ms"):
        if k in m:
            line[k] = m[k]
    wl = m.pop("_wl")

    if not args.no_extra and args.config == "shield":
        # the other configured workloads of the same default run
        blk = measure(api, W, torch, "block", "auto", "cdf", "trilinear", False,
                      args.steps, args.warmup, other_sampler=True)
        blk.pop("_wl")
        if not args.no_gather:
            blk["gather_ceiling"] = gather_ceiling(torch, blk["value"])
        line["block"] = blk
        scan = measure(api, W, torch, "scan", "auto", "cdf", "trilinear", False,
                       args.steps, args.warmup)
        scan.pop("_wl")
        line["scan"] = scan
        line["design_step"] = design_step(api, W, torch)
    elif args.config == "block" and not args.no_gather:
        line["gather_ceiling"] = gather_ceiling(torch, m["value"])

    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_muons or CPU_MUONS[args.config])
    print(json.dumps(line), flush=True)


# Oracle sample of the cpu_baseline leg: about 10 s on 16 host threads.
CPU_MUONS = {"tiny": 10_000, "block": 1_000_000, "shield": 500_000, "scan": 500_000,
             "blocks": 500_000, "logbins": 1_000_000}


def measure(api, W, torch, config, mode_arg, sampler, interp, stage_field, steps, warmup,
            other_sampler=False, block=0, compact=0):
    """Time one workload: every launch form it admits is autotuned and probed,
    the fastest is timed over `steps` passes after `warmup` untimed ones."""
    wl = W.make_workload(config)
    api.load_workload(wl)
    dm = api.DeviceMuons.from_host(wl.muons)
    scales = None
    if wl.run.scales is not None:
        scales = torch.from_numpy(np.ascontiguousarray(wl.run.scales, np.float32)).cuda()
    use_graph = config == "scan"

    def spec_for(mode, smp=sampler):
        return api.RunSpec.from_workload(wl, mode=mode, sampler=smp, interp=interp,
                                         stage_field=stage_field,
                                         use_graph=use_graph and mode != "plain",
                                         block=block, compact_every=compact)

    if mode_arg == "auto":
        modes = ["plain", "persistent"]
        if wl.run.n_variants > 1:
            modes.append("variant_waves")
    else:
        modes = [mode_arg]
    pinned = block > 0 and mode_arg != "auto"
    tuned = {md: api.autotune(dm, spec_for(md), scales=scales)
             for md in modes if md != "plain" and not pinned} or None
    outs = {md: api.alloc_result(spec_for(md), len(dm), "cuda") for md in modes}
    probe = {}
    for md in modes:
        sp = spec_for(md)
        for _ in range(max(1, warmup)):
            api.propagate(dm, sp, scales=scales, out=outs[md])
        _, ms = _time_launches(lambda: api.propagate(dm, sp, scales=scales, out=outs[md]), 2,
                               torch)
        probe[md] = ms
    mode = min(probe, key=probe.get)
    sp = spec_for(mode)
    out = outs[mode]
    for _ in range(warmup):
        api.propagate(dm, sp, scales=scales, out=out)
    torch.cuda.synchronize()
    steps_per_pass = int(out.n_steps.to(torch.int64).sum().item())
    wall, ev_ms = _time_launches(lambda: api.propagate(dm, sp, scales=scales, out=out), steps,
                                 torch)
    value = steps_per_pass * steps / wall
    lanes = int(out.n_steps.numel())
    kernel = {"plain": "k_plain", "persistent": "k_pass",
              "variant_waves": "k_variant_waves"}[mode]
    mix = None
    if config in ("shield", "blocks"):
        mix = step_mix(api, spec_for("plain"), scales, wl)
    ops = algorithmic_ops(config, steps_per_pass, lanes, mode, wl.run.n_variants, mix)
    alg_ops = sum(ops.values())
    achieved = alg_ops / (ev_ms * 1e-3)
    peak = alu_peak(ops)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "Tops/s (VALU lane-ops)", "frac": achieved / peak,
                "traffic": measured_traffic(kernel, config), "kernel": kernel,
                "kernel_ms": ev_ms, "ops_per_pass": alg_ops,
                "ops_mix": {c: v / steps_per_pass for c, v in ops.items()},
                "frac_of_base_issue_rate": achieved / VALU_BASE_LANE_OPS}
    if mix is not None:
        roofline["step_mix_sample"] = mix
    res = {"_wl": wl, "value": value, "ms_per_step": wall / steps * 1e3,
           "config": {"workload": WORKLOADS[config], "muons": len(dm), "lanes": lanes,
                      "muon_steps_per_pass": steps_per_pass, "mode": mode, "sampler": sampler,
                      "interp": interp, "stage_field": stage_field, "mode_probe_ms": probe,
                      "autotune": tuned},
           "roofline": roofline}
    if config == "scan":
        res["per_variant_plain_ms"] = per_variant_plain(api, dm, wl, scales, torch)
    if other_sampler:
        other = "alias" if sampler == "cdf" else "cdf"
        so = spec_for(mode, other)
        oo = api.alloc_result(so, len(dm), "cuda")
        for _ in range(max(1, warmup)):
            api.propagate(dm, so, scales=scales, out=oo)
        torch.cuda.synchronize()
        st = int(oo.n_steps.to(torch.int64).sum().item())
        _, oms = _time_launches(lambda: api.propagate(dm, so, scales=scales, out=oo),
                                max(2, min(steps, 5)), torch)
        res["other_sampler"] = {"sampler": other, "mode": mode, "kernel_ms": oms,
                                "muon_steps_per_pass": st,
                                "muon_steps_per_s": st / (oms * 1e-3)}
    return res


def step_mix(api, spec, scales, wl, n_sample=8192):
    """Fractions of the steps of the first n_sample lanes that are material or
    not, with a field or not, read from the transport's own per-step trace
    (volume and momentum bin; bin -1 = no material).  On the shield every
    step inside the map has a field; on the convex blocks the block's uniform
    field decides."""
    import torch
    n = min(n_sample, len(wl.muons))
    steps_cap = wl.run.max_steps
    sample = api.DeviceMuons.from_host(wl.muons.take(np.arange(n)))
    res = api.propagate(sample, spec, scales=scales, trace_steps=steps_cap, n_trace=n)
    torch.cuda.synchronize()
    tr = res.trace[:n].cpu().numpy()
    ns = res.n_steps[:n].cpu().numpy()
    k = np.arange(steps_cap)[None, :]
    taken = k < ns[:, None]
    vol, mat = tr[:, :, 0], tr[:, :, 1] >= 0
    if wl.field is not None:
        field = np.ones_like(mat)
    else:
        bb = np.zeros((len(wl.geom.material) + 1, 3), np.float32)
        if wl.geom.b_box is not None:
            bb[:-1] = np.asarray(wl.geom.b_box, np.float32)
        field = (bb[vol] != 0).any(axis=-1)          # vol -1 picks the zero last row
    tot = max(int(taken.sum()), 1)
    frac = lambda m: float((taken & m).sum()) / tot
    return {"lanes": n, "steps": tot, "mat_field": frac(mat & field),
            "mat_nofield": frac(mat & ~field), "vac_field": frac(~mat & field),
            "vac_nofield": frac(~mat & ~field)}


def gather_rate(torch, nbytes, width, loads=256, reps=3):
    """Independent uniformly random loads of `width` bytes per second from an
    `nbytes` buffer at full occupancy (libmt_gbench.so)."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2512_10520_amd", "libmt_gbench.so"))
    lib.mtb_gather.argtypes = [C.c_void_p, C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_uint32,
                               C.c_void_p, C.c_void_p]
    buf = torch.randint(0, 2 ** 31 - 1, (nbytes // 4,), dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    blocks = 256 * 8                      # 256 CUs x 8 blocks of 256 threads
    stream = torch.cuda.current_stream().cuda_stream

    def run():
        if lib.mtb_gather(buf.data_ptr(), nbytes, width, loads, blocks, 12345, sink.data_ptr(),
                          stream) != 0:
            raise RuntimeError("gather microbenchmark launch failed")

    run()
    _, ms = _time_launches(run, reps, torch)
    return blocks * 256 * loads / (ms * 1e-3)


# Loop body of each k_valu kind in the gfx950 assembly: 8 instructions of the
# kind (kind 2 also has one v_add_u32 and two v_mov_b32 per iteration).
ALU_KINDS = {0: ("v_fmac_f32", 8), 1: ("v_add_f32", 8), 2: ("v_lshl_add_u32", 11),
             3: ("v_fmac_f64", 8), 4: ("v_mad_u64_u32", 8)}


def alu_rates(torch, iters=4096, clock_hz=2.4e9, simds=1024):
    """SIMD cycles per wave-level instruction of each kind at full occupancy
    (k_valu in libmt_gbench.so): 4 means one 64-lane instruction per 4 cycles
    per 16-lane SIMD."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2512_10520_amd", "libmt_gbench.so"))
    lib.mtb_valu.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint32, C.c_void_p, C.c_void_p]
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    blocks = 256 * 8
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for kind, (name, per_iter) in ALU_KINDS.items():
        def run():
            if lib.mtb_valu(kind, iters, blocks, 7, sink.data_ptr(), stream) != 0:
                raise RuntimeError("VALU microbenchmark launch failed")
        run()
        _, ms = _time_launches(run, 3, torch)
        wave_instr = blocks * 256 / 64 * iters * per_iter
        out[name] = simds * clock_hz * (ms * 1e-3) / wave_instr
    return out


def gather_ceiling(torch, value):
    """The block path's gather roofline: its draw makes about one dependent
    table load per material step (the 8-byte guide entry; a probe of the
    cumulative counts for ~2 % of draws), and its tables are L2-resident in
    practice (99 % L2 hits), so the ceiling is R_gather at an L2-resident
    buffer of 3.6 MiB (one material's cumulative counts) divided by 1.02
    gathers per step."""
    nbytes = 3774874
    r4 = gather_rate(torch, nbytes, 4)
    gathers_per_step = 1.02
    ceiling = r4 / gathers_per_step
    # The method's own gathers: a binary search over the 10^4 cumulative
    # counts of a histogram is 14 dependent probes per material step.
    search_gathers = 14
    return {"r_gather_loads_per_s": r4, "buffer_bytes": nbytes, "load_bytes": 4,
            "gathers_per_step": gathers_per_step, "ceiling_muon_steps_per_s": ceiling,
            "frac": value / ceiling, "search_gathers_per_step": search_gathers,
            "frac_of_search_ceiling": value * search_gathers / r4}


def per_variant_plain(api, dm, wl, scales, torch, reps=2):
    """The scan as 64 separate plain launches (one per field-scale variant),
    the form a caller without the batched launch would use."""
    v = wl.run.n_variants
    spec = api.RunSpec.from_workload(wl, mode="plain")
    spec.n_variants = 1
    out = api.alloc_result(spec, len(dm), "cuda")
    rows = [scales[i:i + 1].contiguous() for i in range(v)]

    def one_scan():
        for i in range(v):
            api.propagate(dm, spec, scales=rows[i], out=out)

    one_scan()
    _, ms = _time_launches(one_scan, reps, torch)
    return ms


def algorithmic_ops(config, steps, lanes, mode="plain", n_variants=64, mix=None):
    """Algorithmic operations of one pass by class (see OPS).  block/scan/diff/
    logbins: the first step of every muon starts in vacuum before the box;
    tiny: zero field.  shield and blocks: the material / field split of the
    steps (`mix`, fractions from step_mix) weights the step kinds; every
    shield step looks up the map.  The variant-wave form shares the Philox
    block of a material step among share_group(n_variants) lanes."""
    scale = lambda k, parts: [(k * c, key) for c, key in parts]
    if config in ("block", "scan", "diff", "logbins"):
        n_mat = steps - lanes
        out = _ops(*scale(n_mat, [(1, "material")]), (lanes, "vacuum"))
    elif config == "tiny":
        n_mat = steps - lanes
        out = _ops(*scale(n_mat, [(1, "material"), (1, "straight")]), (lanes, "vacuum"))
    else:
        if mix is None:
            mix = {"mat_field": 1.0, "mat_nofield": 0.0, "vac_field": 0.0, "vac_nofield": 0.0}
        look = "map" if config == "shield" else "block_lookup"
        n_mat = steps * (mix["mat_field"] + mix["mat_nofield"])
        out = _ops(*scale(steps * mix["mat_field"], [(1, "material"), (1, look)]),
                   *scale(steps * mix["mat_nofield"], [(1, "material"), (1, "straight"),
                                                       (1, look)]),
                   *scale(steps * mix["vac_field"], [(1, "field_step"), (1, look)]),
                   *scale(steps * mix["vac_nofield"], [(1, "vacuum"), (1, look)]))
    if mode == "variant_waves":
        keep = 1.0 / share_group(n_variants)
        for c, v in PHILOX.items():
            out[c] -= n_mat * v * (1.0 - keep)
    return out


def measured_traffic(kernel, config):
    """HBM bytes per launch of this kernel on this workload, from the counter
    summary under profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a plain copy
    of known size), or None if there is none or the kernel source changed
    since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{config}_counters.md")
    src = os.path.join(ROOT, "paper_2512_10520_amd", "csrc", "mt_kernels.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and " = " in line:
            k, v = line[2:].split(" = ", 1)
            fields[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def design_step(api, W, torch, reps=3):
    """Differentiable form at 10^6 muons: forward with checkpoints, loss, and
    the adjoint back to initial states and field scales."""
    wl = W.make_workload("diff")
    api.load_workload(wl)
    dm = api.DeviceMuons.from_host(wl.muons)
    spec = api.RunSpec.from_workload(wl)
    scales = torch.from_numpy(np.ascontiguousarray(wl.run.scales, np.float32)).cuda()
    plain = api.alloc_result(spec, len(dm), "cuda")
    ex = wl.extra
    fwd_ms, ck_ms, bwd_ms = [], [], []
    for r in range(reps + 1):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        x0 = dm.state.clone().requires_grad_(True)
        sc = scales.clone().requires_grad_(True)
        e[0].record()
        api.propagate(dm, spec, scales=scales, out=plain)
        e[1].record()
        st, status, _ = api.transport(x0, sc, dm.q, spec)
        loss = api.detector_loss(st, status, ex["z_det"], ex["r_ap"], ex["r_scale"])
        e[2].record()
        loss.backward()
        e[3].record()
        torch.cuda.synchronize()
        if r > 0:
            fwd_ms.append(e[0].elapsed_time(e[1]))
            ck_ms.append(e[1].elapsed_time(e[2]))
            bwd_ms.append(e[2].elapsed_time(e[3]))
    f, c, b = (float(np.median(v)) for v in (fwd_ms, ck_ms, bwd_ms))
    steps = int(plain.n_steps.to(torch.int64).sum().item())
    # The adjoint kernel alone: without a scale gradient the backward call
    # launches nothing else.
    fwd = api.propagate(dm, spec, scales=scales, ckpt=True)
    g_out = torch.ones((6, len(dm)), dtype=torch.float64, device="cuda")
    api.propagate_backward(dm, spec, fwd, g_out, scales=scales)
    _, adj_ms = _time_launches(lambda: api.propagate_backward(dm, spec, fwd, g_out, scales=scales),
                               reps, torch)
    n_mag = int(np.asarray(wl.run.scales).shape[-1])
    alg = adjoint_bytes(steps, len(dm), n_mag)
    achieved = alg / (adj_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("k_adjoint", "diff"),
                "kernel": "k_adjoint", "kernel_ms": adj_ms, "bytes_per_pass": alg}
    return {"workload": "diff: 8 iron slabs at unit scale, 10^6 muons, loss at z = 30 m",
            "muon_steps_per_pass": steps,
            "forward_ms": f, "forward_ckpt_ms": c, "backward_ms": b,
            "design_step_ms": c + b, "backward_over_forward": b / f,
            "adjoint_roofline": roofline,
            "grad_scales": sc.grad.cpu().tolist()}


HBM_PEAK_GBS = 8000.0


def adjoint_bytes(steps, lanes, n_mag):
    """Device-memory bytes the checkpoint-and-replay adjoint has to move.  Per
    muon-step: the 12-byte kick record read twice (segment replay and reverse
    sweep), the 12-byte pre-kick momentum written in the replay and read in
    the reverse sweep, and a 48-byte FP64 checkpoint read once per 16 steps
    (the step's volume is found again by the replay and kept in LDS).
    Per lane: the output gradient read and the input gradient written (48
    bytes each), step count, status and charge (16), and one FP64 scale
    gradient per magnet written."""
    return steps * (2 * 12 + 2 * 12 + 48 / 16) + lanes * (48 + 48 + 16 + 8 * n_mag)


def cpu_baseline(wl, n_muons):
    import oracle
    idx = np.arange(min(n_muons, len(wl.muons)))
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    res = oracle.propagate(wl, idx)
    dt = time.perf_counter() - t0
    steps = int(res.n_steps.astype(np.int64).sum())
    return {"value": steps / dt, "unit": "muon-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {len(idx)} muons of the same workload ({steps} muon-steps, "
                      f"{dt:.1f} s wall, FP64, OpenMP dynamic schedule)"}


if __name__ == "__main__":
    main()
