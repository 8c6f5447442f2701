"""Python binding of the C ABI: argument marshalling between torch tensors
(device memory, streams) and libmt.so.  Every transport step runs in the HIP
kernels; nothing here computes any part of the method.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import MtMuons, MtParams, MtResult, check

MODES = {"plain": _lib.MT_MODE_PLAIN, "persistent": _lib.MT_MODE_PERSISTENT,
         "variant_waves": _lib.MT_MODE_VARIANT_WAVES}
SAMPLERS = {"cdf": _lib.MT_SAMPLER_CDF, "alias": _lib.MT_SAMPLER_ALIAS}
SAMPLER_NAMES = {v: k for k, v in SAMPLERS.items()}
INTERPS = {"trilinear": _lib.MT_INTERP_TRILINEAR, "nearest": _lib.MT_INTERP_NEAREST}
INTERP_NAMES = {v: k for k, v in INTERPS.items()}


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream_handle(stream: Optional[torch.cuda.Stream]):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


# ---------------------------------------------------------------------------
# Loaders (host arrays in, library-owned device tables)
# ---------------------------------------------------------------------------
def load_histograms(hist) -> None:
    """Load a ``workloads.Histograms`` (or any object with the same fields)."""
    L = _lib.load()
    edges = _host(hist.p_edges, np.float64)
    counts = _host(hist.counts, np.uint32)
    n_mat, n_pbin, n_loss, n_scat = counts.shape
    la = getattr(hist, "log_axes", (False, False))
    axes = (_lib.MT_AXIS_LOG_LOSS if la[0] else 0) | (_lib.MT_AXIS_LOG_SCAT if la[1] else 0)
    check(L.mt_load_histograms_ex(n_mat, n_pbin, edges.ctypes.data, n_loss,
                                  float(hist.loss_lo), float(hist.loss_hi), n_scat,
                                  float(hist.scat_lo), float(hist.scat_hi), counts.ctypes.data,
                                  axes))


def optimal_edges(p_probe, phi, eps: float, max_edges: int = 4096) -> np.ndarray:
    """Bounded-variation momentum binning (``mt_optimal_edges``, host code)."""
    L = _lib.load()
    p = _host(p_probe, np.float64)
    f = _host(phi, np.float64)
    out = np.zeros(max_edges, np.float64)
    n = C.c_int32(0)
    check(L.mt_optimal_edges(p.ctypes.data, f.ctypes.data, len(p), float(eps), out.ctypes.data,
                             int(max_edges), C.byref(n)))
    return out[:n.value].copy()


_loaded = {"n_mag": 0}


def load_geometry(geom) -> None:
    """Load a ``workloads.Geometry``: boxes (``mt_load_geometry``) or, when
    ``geom.poly`` is set, convex blocks (``mt_load_blocks``)."""
    L = _lib.load()
    mat = _host(geom.material, np.int32)
    bb = None if geom.b_box is None else _host(geom.b_box, np.float32)
    mag = None if geom.magnet is None else _host(geom.magnet, np.int32)
    world = _host(geom.world, np.float64)
    bbp = None if bb is None else bb.ctypes.data
    magp = None if mag is None else mag.ctypes.data
    if getattr(geom, "poly", None) is not None:
        blk = _host(geom.poly, np.float64).reshape(-1, 18)
        check(L.mt_load_blocks(len(mat), blk.ctypes.data, mat.ctypes.data, bbp, magp,
                               int(geom.n_mag), world.ctypes.data))
    else:
        box = _host(geom.box, np.float64).reshape(-1, 6)
        check(L.mt_load_geometry(len(mat), box.ctypes.data, mat.ctypes.data, bbp, magp,
                                 int(geom.n_mag), world.ctypes.data))
    _loaded["n_mag"] = int(geom.n_mag)


def load_field(fmap) -> None:
    """Load a ``workloads.FieldMap``; ``None`` unloads the map."""
    L = _lib.load()
    if fmap is None:
        check(L.mt_load_field(0, 0, 0, None, None, None))
        return
    b = _host(fmap.b, np.float32)
    nz, ny, nx, _ = b.shape
    lo, hi = _host(fmap.lo, np.float64), _host(fmap.hi, np.float64)
    check(L.mt_load_field(nx, ny, nz, lo.ctypes.data, hi.ctypes.data, b.ctypes.data))


def load_workload(wl) -> None:
    load_histograms(wl.hist)
    load_geometry(wl.geom)
    load_field(wl.field)


OPTIONS = {"guide_bits": _lib.MT_OPT_GUIDE_BITS, "adjoint_block": _lib.MT_OPT_ADJOINT_BLOCK,
           "adjoint_lds_history": _lib.MT_OPT_ADJOINT_LDS_HISTORY}
OPTION_DEFAULTS = {"guide_bits": 0, "adjoint_block": 64, "adjoint_lds_history": 0}


def set_option(name: str, value: int) -> None:
    """Set a tuning switch (``mt_set_option``); none changes a result."""
    check(_lib.load().mt_set_option(OPTIONS[name], int(value)))


def last_error() -> str:
    return _lib.load().mt_last_error().decode(errors="replace")


def release() -> None:
    _lib.load().mt_release()


def device_info() -> dict:
    info = np.zeros(4, np.int32)
    check(_lib.load().mt_device_info(info.ctypes.data))
    return {"compute_units": int(info[0]), "xcds": int(info[1]), "lds_per_block": int(info[2]),
            "wave_size": int(info[3])}


# ---------------------------------------------------------------------------
# Device muon states
# ---------------------------------------------------------------------------
@dataclass
class DeviceMuons:
    """SoA muon states on the GPU: state [6][n] float64 (x, y, z, px, py, pz)
    and charges [n] int8."""

    state: torch.Tensor
    q: torch.Tensor

    def __len__(self) -> int:
        return int(self.state.shape[1])

    @staticmethod
    def from_host(m, device="cuda") -> "DeviceMuons":
        st = torch.from_numpy(np.array(m.stacked(), dtype=np.float64, order="C")).to(device)
        q = torch.from_numpy(np.array(m.q, dtype=np.int8, order="C")).to(device)
        return DeviceMuons(st.contiguous(), q.contiguous())

    def c_struct(self) -> MtMuons:
        s = self.state
        return MtMuons(*[s[a].data_ptr() for a in range(6)], self.q.data_ptr())


@dataclass
class Result:
    state: torch.Tensor          # [6][lanes] float64
    status: torch.Tensor         # [lanes] int32
    n_steps: torch.Tensor        # [lanes] int32
    volume: torch.Tensor         # [lanes] int32
    trace: Optional[torch.Tensor] = None   # [n_trace][trace_steps][3] int32
    ckpt: Optional[torch.Tensor] = None    # [n_ckpt][6][lanes] float64
    tape: Optional[torch.Tensor] = None    # [max_steps][lanes][3] float32
    tally: Optional[torch.Tensor] = None   # [n_variants][3] float64


@dataclass
class RunSpec:
    step: float
    max_steps: int
    p_min: float
    seed: int = 0
    n_variants: int = 1
    mode: str = "plain"
    block: int = 0
    compact_every: int = 0
    use_graph: bool = False
    sampler: str = "cdf"           # "cdf" (inverse CDF) or "alias"
    interp: str = "trilinear"      # field map lookup: "trilinear" or "nearest"
    stage_field: bool = False      # evaluate the field at every RK4 stage

    @staticmethod
    def from_workload(wl, **kw) -> "RunSpec":
        r = wl.run
        kw.setdefault("sampler", SAMPLER_NAMES[getattr(r, "sampler", 0)])
        kw.setdefault("interp", INTERP_NAMES[getattr(r, "interp", 0)])
        kw.setdefault("stage_field", bool(getattr(r, "stage_field", 0)))
        return RunSpec(step=r.step, max_steps=r.max_steps, p_min=r.p_min, seed=r.seed,
                       n_variants=r.n_variants, **kw)


def _params(spec: RunSpec, scales, ckpt=None, tape=None, trace=None, n_trace=0, trace_steps=0,
            tally=None, z_det=0.0, r_ap=0.0, r_scale=0.0) -> MtParams:
    return MtParams(step_m=float(spec.step), max_steps=int(spec.max_steps),
                    p_min=float(spec.p_min), seed=int(spec.seed) & (2 ** 64 - 1),
                    n_variants=int(spec.n_variants), scales=_ptr(scales),
                    mode=MODES[spec.mode], block=int(spec.block),
                    compact_every=int(spec.compact_every), use_graph=int(bool(spec.use_graph)),
                    ckpt_every=_lib.CKPT_EVERY if ckpt is not None else 0, ckpt=_ptr(ckpt),
                    tape=_ptr(tape), trace=_ptr(trace), n_trace=int(n_trace),
                    trace_steps=int(trace_steps), tally=_ptr(tally), z_det=float(z_det),
                    r_ap=float(r_ap), r_scale=float(r_scale), sampler=SAMPLERS[spec.sampler],
                    interp=INTERPS[spec.interp], stage_field=int(bool(spec.stage_field)))


def _check_scales(scales, spec: RunSpec):
    if scales is None:
        return None
    if scales.dtype != torch.float32 or not scales.is_cuda or not scales.is_contiguous():
        raise ValueError("scales must be a contiguous float32 CUDA tensor [n_variants][n_mag]")
    if scales.dim() != 2 or tuple(scales.shape) != (spec.n_variants, _loaded["n_mag"]):
        raise ValueError(f"scales must have shape [n_variants={spec.n_variants}]"
                         f"[n_mag={_loaded['n_mag']}]")
    return scales


def _check_muons(m: DeviceMuons):
    if m.state.dtype != torch.float64 or m.state.dim() != 2 or m.state.shape[0] != 6:
        raise ValueError("muon state must be a float64 tensor of shape [6][n]")
    if not (m.state.is_cuda and m.q.is_cuda):
        raise ValueError("muon tensors must live on the GPU")
    if not m.state.is_contiguous() or not m.q.is_contiguous() or m.q.dtype != torch.int8:
        raise ValueError("muon tensors must be contiguous; charges int8")
    if m.q.shape[0] != m.state.shape[1]:
        raise ValueError("charges and states disagree in length")


def alloc_result(spec: RunSpec, n: int, device, trace_steps=0, n_trace=0, ckpt=False,
                 tally=False) -> Result:
    lanes = n * spec.n_variants
    dev = torch.device(device)
    r = Result(state=torch.empty((6, lanes), dtype=torch.float64, device=dev),
               status=torch.empty(lanes, dtype=torch.int32, device=dev),
               n_steps=torch.empty(lanes, dtype=torch.int32, device=dev),
               volume=torch.empty(lanes, dtype=torch.int32, device=dev))
    if trace_steps > 0 and n_trace > 0:
        r.trace = torch.full((n_trace, trace_steps, 3), -2, dtype=torch.int32, device=dev)
    if ckpt:
        n_ck = max(1, -(-spec.max_steps // _lib.CKPT_EVERY))
        r.ckpt = torch.empty((n_ck, 6, lanes), dtype=torch.float64, device=dev)
        r.tape = torch.empty((max(1, spec.max_steps), lanes, 3), dtype=torch.float32, device=dev)
    if tally:
        r.tally = torch.empty((spec.n_variants, 3), dtype=torch.float64, device=dev)
    return r


def _check_result(out: Result, spec: RunSpec, n: int, ckpt: bool, tally: bool) -> None:
    """Check that preallocated outputs are large enough for this call (the C
    ABI takes raw pointers and cannot check buffer sizes itself)."""
    lanes = n * spec.n_variants
    if tuple(out.state.shape) != (6, lanes) or out.state.dtype != torch.float64:
        raise ValueError(f"result state must be float64 [6][{lanes}]")
    for name in ("status", "n_steps", "volume"):
        t = getattr(out, name)
        if t.numel() != lanes or t.dtype != torch.int32:
            raise ValueError(f"result {name} must be int32 [{lanes}]")
    if out.trace is not None and (out.trace.dim() != 3 or out.trace.shape[2] != 3 or
                                  out.trace.dtype != torch.int32):
        raise ValueError("trace must be int32 [n_trace][trace_steps][3]")
    if ckpt:
        n_ck = max(1, -(-spec.max_steps // _lib.CKPT_EVERY))
        if out.ckpt is None or out.tape is None:
            raise ValueError("checkpointing needs ckpt and tape buffers in the result")
        if (out.ckpt.shape[0] < n_ck or tuple(out.ckpt.shape[1:]) != (6, lanes) or
                out.ckpt.dtype != torch.float64):
            raise ValueError(f"ckpt must be float64 [>={n_ck}][6][{lanes}]")
        if (out.tape.shape[0] < spec.max_steps or tuple(out.tape.shape[1:]) != (lanes, 3) or
                out.tape.dtype != torch.float32):
            raise ValueError(f"tape must be float32 [>={spec.max_steps}][{lanes}][3]")
    if tally and (out.tally is None or tuple(out.tally.shape) != (spec.n_variants, 3)):
        raise ValueError(f"tally must be float64 [{spec.n_variants}][3]")


def propagate(muons: DeviceMuons, spec: RunSpec, scales: Optional[torch.Tensor] = None,
              trace_steps: int = 0, n_trace: int = 0, ckpt: bool = False,
              tally: Optional[dict] = None, out: Optional[Result] = None,
              stream: Optional[torch.cuda.Stream] = None, noalloc: bool = False) -> Result:
    """Transport ``muons`` on the GPU (``mt_propagate``).

    ``tally`` = dict(z_det=..., r_ap=..., r_scale=...) requests per-variant
    detector-plane tallies.  ``out`` reuses preallocated result tensors.
    ``noalloc`` calls ``mt_propagate_noalloc`` instead, which allocates no
    device memory (pass ``out`` as well to allocate nothing here either).
    """
    _check_muons(muons)
    scales = _check_scales(scales, spec)
    n = len(muons)
    if out is None:
        out = alloc_result(spec, n, muons.state.device, trace_steps, n_trace, ckpt,
                           tally is not None)
    _check_result(out, spec, n, ckpt, tally is not None)
    t = tally or {}
    tr_rows, tr_steps = (0, 0) if out.trace is None else tuple(out.trace.shape[:2])
    p = _params(spec, scales, ckpt=out.ckpt if ckpt else None, tape=out.tape if ckpt else None,
                trace=out.trace, n_trace=tr_rows, trace_steps=tr_steps,
                tally=out.tally if tally is not None else None, z_det=t.get("z_det", 0.0),
                r_ap=t.get("r_ap", 0.0), r_scale=t.get("r_scale", 0.0))
    res = MtResult(out.status.data_ptr(), out.n_steps.data_ptr(), out.volume.data_ptr())
    o = MtMuons(*[out.state[a].data_ptr() for a in range(6)], None)
    i = muons.c_struct()
    L = _lib.load()
    fn = L.mt_propagate_noalloc if noalloc else L.mt_propagate
    check(fn(C.byref(p), n, C.byref(i), C.byref(o), C.byref(res), _stream_handle(stream)))
    return out


def propagate_backward(muons: DeviceMuons, spec: RunSpec, fwd: Result, g_out: torch.Tensor,
                       scales: Optional[torch.Tensor] = None, n_mag: int = 0,
                       stream: Optional[torch.cuda.Stream] = None):
    """Pathwise adjoint (``mt_propagate_backward``) of a checkpointed forward.

    Returns (g_in [6][lanes] float64, g_scales [n_variants][n_mag] float64 or None).
    """
    _check_muons(muons)
    scales = _check_scales(scales, spec)
    if fwd.ckpt is None or fwd.tape is None:
        raise ValueError("the forward result carries no checkpoints: call propagate(ckpt=True)")
    n = len(muons)
    _check_result(fwd, spec, n, True, False)
    lanes = n * spec.n_variants
    g_out = g_out.to(torch.float64).contiguous()
    if tuple(g_out.shape) != (6, lanes):
        raise ValueError(f"g_out must have shape [6][{lanes}]")
    g_in = torch.empty_like(g_out)
    g_scales = (torch.empty((spec.n_variants, n_mag), dtype=torch.float64, device=g_out.device)
                if n_mag > 0 else None)
    p = _params(spec, scales, ckpt=fwd.ckpt, tape=fwd.tape)
    res = MtResult(fwd.status.data_ptr(), fwd.n_steps.data_ptr(), fwd.volume.data_ptr())
    i = muons.c_struct()
    check(_lib.load().mt_propagate_backward(C.byref(p), n, C.byref(i), C.byref(res),
                                            g_out.data_ptr(), g_in.data_ptr(), _ptr(g_scales),
                                            _stream_handle(stream)))
    return g_in, g_scales


def autotune(muons: DeviceMuons, spec: RunSpec, scales=None, out: Optional[Result] = None,
             stream=None):
    """Time the candidate (block, steps per pass) pairs of the compacting
    form (mode "persistent") -- or the block sizes of the variant-wave form when ``spec.mode`` is
    "variant_waves" -- on this call and remember the fastest (``mt_autotune``)."""
    _check_muons(muons)
    scales = _check_scales(scales, spec)
    n = len(muons)
    if out is None:
        out = alloc_result(spec, n, muons.state.device)
    p = _params(spec, scales)
    if spec.mode != "variant_waves":
        p.mode = _lib.MT_MODE_PERSISTENT
    res = MtResult(out.status.data_ptr(), out.n_steps.data_ptr(), out.volume.data_ptr())
    o = MtMuons(*[out.state[a].data_ptr() for a in range(6)], None)
    i = muons.c_struct()
    bb, bc, ms = C.c_int32(0), C.c_int32(0), C.c_float(0)
    check(_lib.load().mt_autotune(C.byref(p), n, C.byref(i), C.byref(o), C.byref(res),
                                  _stream_handle(stream), C.byref(bb), C.byref(bc), C.byref(ms)))
    return {"block": bb.value, "compact_every": bc.value, "ms": ms.value}


# ---------------------------------------------------------------------------
# Differentiable form
# ---------------------------------------------------------------------------
class Transport(torch.autograd.Function):
    """Differentiable transport: (x0 [6][n] float64, scales [V][n_mag] float32)
    -> final states [6][V*n] float64, with status and step counts returned as
    non-differentiable outputs.  The backward pass is the hand-written adjoint
    kernel (pathwise: sampled kicks and all discrete decisions held fixed)."""

    @staticmethod
    def forward(ctx, x0, scales, q, spec: RunSpec):
        m = DeviceMuons(x0.detach().contiguous(), q)
        sc = scales.detach().to(torch.float32).contiguous() if scales is not None else None
        res = propagate(m, spec, scales=sc, ckpt=True)
        ctx.spec = spec
        ctx.muons = m
        ctx.scales = sc
        ctx.res = res
        ctx.scales_dtype = None if scales is None else scales.dtype
        ctx.mark_non_differentiable(res.status, res.n_steps)
        return res.state, res.status, res.n_steps

    @staticmethod
    def backward(ctx, g_state, _g_status=None, _g_steps=None):
        spec = ctx.spec
        n_mag = 0 if ctx.scales is None else int(ctx.scales.shape[1])
        if g_state is None:
            g_state = torch.zeros_like(ctx.res.state)
        g_in, g_sc = propagate_backward(ctx.muons, spec, ctx.res, g_state, scales=ctx.scales,
                                        n_mag=n_mag)
        n = len(ctx.muons)
        g_x0 = g_in.view(6, spec.n_variants, n).sum(dim=1) if spec.n_variants > 1 else g_in
        g_scales = None
        if ctx.needs_input_grad[1] and g_sc is not None:
            g_scales = g_sc.to(ctx.scales_dtype)
        return (g_x0 if ctx.needs_input_grad[0] else None), g_scales, None, None


def transport(x0: torch.Tensor, scales: Optional[torch.Tensor], q: torch.Tensor, spec: RunSpec):
    return Transport.apply(x0, scales, q, spec)


def detector_loss(state: torch.Tensor, status: torch.Tensor, z_det: float = 30.0,
                  r_ap: float = 1.0, r_scale: float = 0.01) -> torch.Tensor:
    """Sum of sigmoid((r_ap - r)/r_scale) over muons that left through z_max,
    r being the radius at z = z_det reached on a straight line (torch ops, so
    autograd supplies dL/d(final state) for the adjoint)."""
    x, y, z, px, py, pz = state
    ok = status == _lib.ST_ZMAX
    dz = z_det - z
    xd = x + dz * px / pz
    yd = y + dz * py / pz
    r = torch.sqrt(xd * xd + yd * yd)
    term = torch.sigmoid((r_ap - r) / r_scale)
    return torch.where(ok, term, torch.zeros_like(term)).sum()
