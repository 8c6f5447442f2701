"""FP64 CPU oracle (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It wraps ``oracle.c`` (plain C, double precision, OpenMP over
muons) through ctypes and adds the detector-plane loss and central finite
differences in numpy.  Nothing here imports the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np
from scipy import special

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

KAPPA = 0.299792458  # GeV / (c T m)

ST_PMIN, ST_ZMAX, ST_XMAX, ST_YMAX, ST_STEPS, ST_INVALID = 1, 2, 3, 4, 5, 6


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("n_mat", C.c_int32), ("n_pbin", C.c_int32), ("n_loss", C.c_int32), ("n_scat", C.c_int32),
        ("p_edges", C.c_void_p),
        ("loss_lo", C.c_double), ("loss_hi", C.c_double),
        ("scat_lo", C.c_double), ("scat_hi", C.c_double),
        ("counts", C.c_void_p),
        ("n_box", C.c_int32),
        ("box", C.c_void_p),
        ("n_poly", C.c_int32), ("poly", C.c_void_p),
        ("material", C.c_void_p), ("b_box", C.c_void_p),
        ("magnet", C.c_void_p),
        ("n_mag", C.c_int32),
        ("world", C.c_double * 3),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("map_lo", C.c_double * 3), ("map_hi", C.c_double * 3),
        ("map", C.c_void_p),
        ("step", C.c_double), ("max_steps", C.c_int32), ("p_min", C.c_double),
        ("seed", C.c_uint64),
        ("scales", C.c_void_p),
        ("sampler", C.c_int32),
        ("log_loss", C.c_int32), ("log_scat", C.c_int32),
        ("interp", C.c_int32),
        ("stage_field", C.c_int32),
    ]


class _In(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "px", "py", "pz", "q", "ids", "variant")]


class _Out(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "px", "py", "pz",
                                          "status", "n_steps", "volume",
                                          "margin_pos", "margin_p", "trace")] + \
               [("trace_steps", C.c_int32), ("kicks", C.c_void_p), ("kick_steps", C.c_int32),
                ("step_margin", C.c_void_p), ("digest", C.c_void_p)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            L.oracle_philox.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
            L.oracle_cdf_build.argtypes = [C.c_void_p, C.c_int64, C.c_void_p]
            L.oracle_cdf_build.restype = C.c_int
            L.oracle_cdf_t.argtypes = [C.c_uint32, C.c_uint32]
            L.oracle_cdf_t.restype = C.c_uint32
            L.oracle_cdf_cell.argtypes = [C.c_void_p, C.c_int64, C.c_uint32]
            L.oracle_cdf_cell.restype = C.c_int64
            L.oracle_alias_build.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
            L.oracle_alias_build.restype = C.c_int
            L.oracle_alias_cell.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_uint32,
                                            C.c_void_p]
            L.oracle_alias_cell.restype = C.c_int64
            L.oracle_rotate.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
            L.oracle_rk4.argtypes = [C.c_void_p, C.c_double, C.c_void_p, C.c_double, C.c_void_p]
            L.oracle_lookup.argtypes = [C.POINTER(_Problem), C.c_void_p]
            L.oracle_lookup.restype = C.c_int32
            L.oracle_poly_inside.argtypes = [C.c_void_p, C.c_void_p]
            L.oracle_poly_inside.restype = C.c_int32
            L.oracle_pbin.argtypes = [C.POINTER(_Problem), C.c_double]
            L.oracle_pbin.restype = C.c_int32
            L.oracle_trilinear.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p]
            L.oracle_nearest.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p]
            for name in ("oracle_geom_margin", "oracle_map_margin"):
                getattr(L, name).argtypes = [C.POINTER(_Problem), C.c_void_p]
                getattr(L, name).restype = C.c_double
            L.oracle_break_margin.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_double,
                                              C.POINTER(C.c_double)]
            L.oracle_break_margin.restype = C.c_double
            L.oracle_bin_margin.argtypes = [C.POINTER(_Problem), C.c_int32, C.c_double]
            L.oracle_bin_margin.restype = C.c_double
            L.oracle_propagate.argtypes = [C.POINTER(_Problem), C.c_int64, C.POINTER(_In),
                                           C.POINTER(_Out), C.c_int32]
            L.oracle_propagate.restype = C.c_int
            L.oracle_max_threads.restype = C.c_int
            _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class Problem:
    """Owns contiguous copies of a workload's tables and the ctypes struct."""

    def __init__(self, wl, scales: Optional[np.ndarray] = None, seed: Optional[int] = None):
        h, g, f, r = wl.hist, wl.geom, wl.field, wl.run
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        P = _Problem()
        P.n_mat, P.n_pbin, P.n_loss, P.n_scat = h.n_mat, h.n_pbin, h.n_loss, h.n_scat
        P.p_edges = _ptr(keep(h.p_edges, np.float64))
        P.loss_lo, P.loss_hi, P.scat_lo, P.scat_hi = h.loss_lo, h.loss_hi, h.scat_lo, h.scat_hi
        P.counts = _ptr(keep(h.counts, np.uint32))
        poly = getattr(g, "poly", None)
        if poly is not None:
            P.n_box, P.box = 0, None
            P.n_poly = len(g.material)
            P.poly = _ptr(keep(np.asarray(poly).reshape(-1, 18), np.float64))
        else:
            P.n_box = len(g.material)
            P.box = _ptr(keep(g.box, np.float64))
            P.n_poly, P.poly = 0, None
        P.material = _ptr(keep(g.material, np.int32))
        P.b_box = _ptr(keep(g.b_box, np.float32))
        P.magnet = _ptr(keep(g.magnet, np.int32))
        P.n_mag = g.n_mag
        P.world = (C.c_double * 3)(*[float(v) for v in g.world])
        if f is not None:
            nx, ny, nz = f.shape_xyz
            P.nx, P.ny, P.nz = nx, ny, nz
            P.map_lo = (C.c_double * 3)(*[float(v) for v in f.lo])
            P.map_hi = (C.c_double * 3)(*[float(v) for v in f.hi])
            P.map = _ptr(keep(f.b, np.float32))
        else:
            P.nx = P.ny = P.nz = 0
            P.map = None
        P.step, P.max_steps, P.p_min = r.step, r.max_steps, r.p_min
        P.seed = r.seed if seed is None else seed
        sc = r.scales if scales is None else scales
        P.scales = None if sc is None else _ptr(keep(sc, np.float64))
        P.sampler = int(getattr(r, "sampler", 0))
        la = getattr(h, "log_axes", (False, False))
        P.log_loss, P.log_scat = int(bool(la[0])), int(bool(la[1]))
        P.interp = int(getattr(r, "interp", 0))
        P.stage_field = int(getattr(r, "stage_field", 0))
        self.struct = P


@dataclass
class Result:
    state: np.ndarray        # float64 [6][n]: x, y, z, px, py, pz
    status: np.ndarray       # int32 [n]
    n_steps: np.ndarray      # int32 [n]
    volume: np.ndarray       # int32 [n]
    margin_pos: np.ndarray   # float64 [n] (m)
    margin_p: np.ndarray     # float64 [n] (relative)
    trace: Optional[np.ndarray] = None   # int32 [n][trace_steps][3]
    kicks: Optional[np.ndarray] = None   # float32 [n][kick_steps][3]
    step_margin: Optional[np.ndarray] = None   # float64 [n][trace_steps+1][2]
    digest: Optional[np.ndarray] = None   # uint64 [n]: FNV-1a of the whole (vol, bin, cell) trace


def propagate(wl, idx=None, variant=None, muons=None, scales=None, seed=None,
              trace_steps: int = 0, kick_steps: int = 0, n_threads: int = 0,
              margins: bool = True, digest: bool = False) -> Result:
    """Run the oracle on muons ``idx`` of the workload (default: all).

    ``idx`` doubles as the Philox muon index of each muon.  ``variant`` gives
    each muon's field-scale variant (default 0).  ``muons`` optionally replaces
    the initial states (a [6][n] float64 array plus charges from the workload)
    while keeping the Philox indices, which is how finite differences on
    common random numbers are formed.  ``margins=False`` skips the decision
    margins (margin_pos / margin_p come back as infinity, step_margin None).
    ``digest=True`` adds a 64-bit hash of each muon's whole (volume, bin,
    cell) step sequence, which compares decision paths without storing them.
    """
    L = lib()
    m = wl.muons
    if idx is None:
        idx = np.arange(len(m), dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    n = len(idx)
    if muons is None:
        st = np.stack([m.x[idx], m.y[idx], m.z[idx], m.px[idx], m.py[idx], m.pz[idx]])
    else:
        st = np.asarray(muons, dtype=np.float64)
    st = np.ascontiguousarray(st, dtype=np.float64)
    q = np.ascontiguousarray(m.q[idx], dtype=np.int8)
    var = None if variant is None else np.ascontiguousarray(
        np.broadcast_to(np.asarray(variant, dtype=np.int32), (n,)))
    prob = Problem(wl, scales=scales, seed=seed)
    out_state = np.zeros((6, n), dtype=np.float64)
    status = np.zeros(n, np.int32)
    nst = np.zeros(n, np.int32)
    vol = np.zeros(n, np.int32)
    mpos = np.zeros(n, np.float64)
    mp = np.zeros(n, np.float64)
    trace = np.full((n, trace_steps, 3), -2, np.int32) if trace_steps > 0 else None
    kicks = np.zeros((n, kick_steps, 3), np.float32) if kick_steps > 0 else None
    smarg = np.full((n, trace_steps + 1, 2), np.inf) if trace_steps > 0 and margins else None
    dig = np.zeros(n, np.uint64) if digest else None
    if not margins:
        mpos[:] = np.inf
        mp[:] = np.inf
    I = _In(*[st[a].ctypes.data for a in range(6)], q.ctypes.data, idx.ctypes.data, _ptr(var))
    O = _Out(*[out_state[a].ctypes.data for a in range(6)], status.ctypes.data, nst.ctypes.data,
             vol.ctypes.data, mpos.ctypes.data if margins else None,
             mp.ctypes.data if margins else None, _ptr(trace), trace_steps,
             _ptr(kicks), kick_steps, _ptr(smarg), _ptr(dig))
    rc = L.oracle_propagate(C.byref(prob.struct), n, C.byref(I), C.byref(O), int(n_threads))
    if rc != 0:
        raise RuntimeError(f"oracle_propagate failed with code {rc}")
    return Result(out_state, status, nst, vol, mpos, mp, trace, kicks, smarg, dig)


# --------------------------------------------------------------------------
# Unit functions (for pin tests)
# --------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().oracle_philox(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def cdf_cells(counts: np.ndarray, t_values: np.ndarray) -> np.ndarray:
    counts = np.ascontiguousarray(counts, dtype=np.uint32).ravel()
    K = counts.size
    cdf = np.zeros(K, np.uint32)
    if lib().oracle_cdf_build(counts.ctypes.data, K, cdf.ctypes.data) != 0:
        raise ValueError("empty or oversized histogram")
    return np.array([lib().oracle_cdf_cell(cdf.ctypes.data, K, int(t)) for t in t_values],
                    dtype=np.int64)


def alias_tables(counts: np.ndarray):
    """Walker Prob/Alias tables of one histogram: (prob uint32 [K], alias
    int32 [K]), prob in units of the histogram total."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32).ravel()
    K = counts.size
    prob = np.zeros(K, np.uint32)
    alias = np.zeros(K, np.int32)
    rc = lib().oracle_alias_build(counts.ctypes.data, K, prob.ctypes.data, alias.ctypes.data)
    if rc != 0:
        raise ValueError("empty or oversized histogram" if rc == -1 else "out of memory")
    return prob, alias


def alias_cell(prob: np.ndarray, alias: np.ndarray, total: int, words) -> int:
    """Cell drawn by the alias method from one Philox block (4 words)."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    return int(lib().oracle_alias_cell(prob.ctypes.data, alias.ctypes.data, prob.size,
                                       int(total), w.ctypes.data))


def cdf_t(w: int, total: int) -> int:
    return int(lib().oracle_cdf_t(int(w), int(total)))


def rotate(p, dp) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    dp = np.ascontiguousarray(dp, dtype=np.float64)
    o = np.zeros(3)
    lib().oracle_rotate(p.ctypes.data, dp.ctypes.data, o.ctypes.data)
    return o


def rk4(y, q, B, h) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    o = np.zeros(6)
    lib().oracle_rk4(y.ctypes.data, float(q), B.ctypes.data, float(h), o.ctypes.data)
    return o


def lookup(wl, r) -> int:
    prob = Problem(wl)
    r = np.ascontiguousarray(r, dtype=np.float64)
    return int(lib().oracle_lookup(C.byref(prob.struct), r.ctypes.data))


def poly_inside(block, r) -> bool:
    """Is r inside one block (float64 [18]: z_lo, z_hi, bottom quad, top quad)?"""
    b = np.ascontiguousarray(block, dtype=np.float64).ravel()
    r = np.ascontiguousarray(r, dtype=np.float64)
    return bool(lib().oracle_poly_inside(b.ctypes.data, r.ctypes.data))


def pbin(wl, pm: float) -> int:
    prob = Problem(wl)
    return int(lib().oracle_pbin(C.byref(prob.struct), float(pm)))


def trilinear(wl, r) -> np.ndarray:
    prob = Problem(wl)
    r = np.ascontiguousarray(r, dtype=np.float64)
    o = np.zeros(3)
    lib().oracle_trilinear(C.byref(prob.struct), r.ctypes.data, o.ctypes.data)
    return o


def nearest(wl, r) -> np.ndarray:
    prob = Problem(wl)
    r = np.ascontiguousarray(r, dtype=np.float64)
    o = np.zeros(3)
    lib().oracle_nearest(C.byref(prob.struct), r.ctypes.data, o.ctypes.data)
    return o


class Decisions:
    """The oracle's discrete decisions and their margins for one workload
    (tables copied once, for many queries)."""

    def __init__(self, wl):
        self._prob = Problem(wl)
        self._p = C.byref(self._prob.struct)
        self._L = lib()

    @staticmethod
    def _r(r):
        return np.ascontiguousarray(r, dtype=np.float64)

    def lookup(self, r) -> int:
        r = self._r(r)
        return int(self._L.oracle_lookup(self._p, r.ctypes.data))

    def geom_margin(self, r) -> float:
        r = self._r(r)
        return float(self._L.oracle_geom_margin(self._p, r.ctypes.data))

    def map_margin(self, r) -> float:
        r = self._r(r)
        return float(self._L.oracle_map_margin(self._p, r.ctypes.data))

    def break_margin(self, r, pm):
        """(position margin in m, momentum margin relative to pm)."""
        r = self._r(r)
        mp = C.c_double(0.0)
        mpos = self._L.oracle_break_margin(self._p, r.ctypes.data, float(pm), C.byref(mp))
        return float(mpos), float(mp.value)

    def bin_margin(self, ibin: int, pm: float) -> float:
        return float(self._L.oracle_bin_margin(self._p, int(ibin), float(pm)))

    def pbin(self, pm: float) -> int:
        return int(self._L.oracle_pbin(self._p, float(pm)))

    def nearest(self, r) -> np.ndarray:
        r = self._r(r)
        o = np.zeros(3)
        self._L.oracle_nearest(self._p, r.ctypes.data, o.ctypes.data)
        return o

    def trilinear(self, r) -> np.ndarray:
        r = self._r(r)
        o = np.zeros(3)
        self._L.oracle_trilinear(self._p, r.ctypes.data, o.ctypes.data)
        return o


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# --------------------------------------------------------------------------
# Optimal momentum binning (appendix "Optimal Momentum Binning")
# --------------------------------------------------------------------------
def optimal_edges(p_probe, phi, eps):
    """Bounded-variation momentum binning on a grid of probe momenta.

    The variation of a candidate bin [p_a, p] is the largest |phi(p') -
    phi(p_a)| over the probes p' in [p_a, p]; the next edge after p_a is the
    supremum of the p for which it stays within eps.  On the probe grid that
    supremum is the first probe whose estimate differs from phi(p_a) by more
    than eps (every p below it passes, it fails), or the last probe.
    Returns the edges p_0 = p_probe[0] < ... < p_N = p_probe[-1].
    """
    p = np.asarray(p_probe, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    edges = [p[0]]
    a = 0
    while a < len(p) - 1:
        nxt = len(p) - 1
        for j in range(a + 1, len(p)):
            if abs(phi[j] - phi[a]) > eps:
                nxt = j
                break
        edges.append(p[nxt])
        a = nxt
    return np.array(edges)


# --------------------------------------------------------------------------
# Detector-plane loss and finite differences (differentiable form)
# --------------------------------------------------------------------------
def detector_loss_terms(state: np.ndarray, status: np.ndarray, z_det: float = 30.0,
                        r_ap: float = 1.0, r_scale: float = 0.01) -> np.ndarray:
    """Per-muon sigmoid((r_ap - r)/r_scale) at the plane z = z_det.

    Muons that left through z_max (status 2) are carried to the plane on a
    straight line (the region beyond the last box is field-free vacuum);
    all others contribute zero.
    """
    x, y, z, px, py, pz = state
    with np.errstate(divide="ignore", invalid="ignore"):
        xd = x + (z_det - z) * px / pz
        yd = y + (z_det - z) * py / pz
        rr = np.sqrt(xd * xd + yd * yd)
        term = special.expit((r_ap - rr) / r_scale)
    return np.where(status == ST_ZMAX, term, 0.0)


def fd_scales(wl, idx, h: float = 1e-3, **loss_kw):
    """Central differences of the summed loss w.r.t. each magnet scale.

    Runs two oracle transports per magnet on common random numbers.  Returns
    (grad [n_mag], per-muon flags [n] that mark muons whose decision trace
    differed between any pair of +h/-h runs and were left out of the sums).
    """
    base = np.asarray(wl.run.scales if wl.run.scales is not None
                      else np.ones((1, wl.geom.n_mag)), dtype=np.float64)
    n_mag = wl.geom.n_mag
    idx = np.asarray(idx, dtype=np.int64)
    plus, minus = [], []
    for m in range(n_mag):
        sp, sm = base.copy(), base.copy()
        sp[0, m] += h
        sm[0, m] -= h
        plus.append(propagate(wl, idx, scales=sp, margins=False, digest=True))
        minus.append(propagate(wl, idx, scales=sm, margins=False, digest=True))
    flagged = np.zeros(len(idx), bool)
    for a, b in zip(plus, minus):
        flagged |= (a.n_steps != b.n_steps) | (a.status != b.status)
        flagged |= a.digest != b.digest
    grad = np.zeros(n_mag)
    for m in range(n_mag):
        lp = detector_loss_terms(plus[m].state, plus[m].status, **loss_kw)
        lm = detector_loss_terms(minus[m].state, minus[m].status, **loss_kw)
        grad[m] = np.sum(np.where(flagged, 0.0, (lp - lm) / (2 * h)))
    return grad, flagged


def fd_inputs(wl, idx, h: float = 1e-3, comps=(0, 1, 3, 4, 5), **loss_kw):
    """Central differences of each muon's loss term w.r.t. its initial
    (x, y, z, px, py, pz) components listed in ``comps``.

    Returns (grad [6][n] with zeros for components not listed, flags [n]).
    """
    idx = np.asarray(idx, dtype=np.int64)
    m = wl.muons
    st0 = np.stack([m.x[idx], m.y[idx], m.z[idx], m.px[idx], m.py[idx], m.pz[idx]])
    grad = np.zeros((6, len(idx)))
    flagged = np.zeros(len(idx), bool)
    for a in comps:
        sp, sm = st0.copy(), st0.copy()
        sp[a] += h
        sm[a] -= h
        rp = propagate(wl, idx, muons=sp, margins=False, digest=True)
        rm = propagate(wl, idx, muons=sm, margins=False, digest=True)
        flagged |= (rp.n_steps != rm.n_steps) | (rp.status != rm.status)
        flagged |= rp.digest != rm.digest
        lp = detector_loss_terms(rp.state, rp.status, **loss_kw)
        lm = detector_loss_terms(rm.state, rm.status, **loss_kw)
        grad[a] = (lp - lm) / (2 * h)
    return grad, flagged
