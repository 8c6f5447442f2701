"""Seeded synthetic inputs for the histogram-sampling muon transport.

This module only *generates inputs*: histogram counts, momentum-bin edges,
box geometries, field maps, incoming muons and field-scale variants.  It holds
none of the transport arithmetic, so both the FP64 CPU oracle and the HIP
library can be fed from it without sharing any of the method's code.

The paper builds its histograms with Geant4 (Section "Building histograms")
and its shield geometry / field map with SHiP-specific tools (Section
"Validation and benchmarking"); none of these are available, so every input
here is a seeded stand-in with the shapes of the five workloads:

``tiny``    1 iron box 1 m long, no field, 32 log momentum bins 1-400 GeV,
            64x64 histograms, 10^4 muons at 100 GeV, charge alternating.
``block``   5 m iron box, uniform 1.7 T along y, 95 log bins 0.18-400 GeV
            (the paper's binning), 100x100 histograms, 10^6 power-law muons.
``shield``  40 axis-aligned boxes (8 stations of iron yokes, an air core and
            concrete walls), 3 materials, trilinear float32 field map
            100x100x300 on 4x4x30 m, 10^7 power-law muons.
``scan``    ``block`` geometry split into 8 iron slabs (one magnet each),
            64 variants of 8 field scales in [0.8, 1.2], 2^17 muons shared by
            all variants.
``diff``    ``scan`` geometry at unit scales with the 10^6 ``block`` muons;
            used for the differentiable (adjoint) form.
``logbins`` ``block`` geometry and muons with the paper's histogram
            parameterisation: both axes binned in log10 (f in [1e-6, 1],
            tau in [1e-6, 0.5]), 95 log momentum bins.
``blocks``  the ``shield`` stations as 40 convex blocks: yokes and air core
            taper along z (seeded per station), the walls stay prisms;
            uniform per-block fields (yokes +-B_m along y, one magnet per
            station), the ``shield`` histograms, 10^6 power-law muons.

Every random draw comes from ``np.random.default_rng([2512, 10520, cfg,
part, ...])`` with its own stream per array, so a prefix of the muon list is
exactly the list generated with a smaller count.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy import special

CONFIGS = ("tiny", "block", "shield", "scan", "diff", "blocks", "logbins")
_CFG_CODE = {"tiny": 1, "block": 2, "shield": 3, "scan": 4, "diff": 5, "blocks": 6,
             "logbins": 7}

# Part codes of the seed sequence.
_PART_HIST, _PART_MUONS, _PART_GEOM, _PART_FIELD, _PART_VARIANTS = 0, 1, 2, 3, 4

# Materials of the recipe: (loss constant a_M [GeV/m], radiation length X0 [m]).
# These shape the synthetic histograms only; they are recipe constants.
MATERIALS = {
    "iron": (1.14, 0.01757),
    "concrete": (0.39, 0.1155),
    "air": (2.2e-4, 303.9),
}


def _rng(*codes: int) -> np.random.Generator:
    return np.random.default_rng([2512, 10520, *codes])


# --------------------------------------------------------------------------
# Histograms
# --------------------------------------------------------------------------
@dataclass
class Histograms:
    """Count histograms H[M][i] over (fractional loss f, transverse kick tau).

    ``counts[m, i, a, b]`` counts muons of material ``m`` and momentum bin ``i``
    whose loss fell in bin ``a`` of [loss_lo, loss_hi] and whose kick fell in
    bin ``b`` of [scat_lo, scat_hi].  Bins are uniform in the value, or in its
    base-10 logarithm on an axis marked in ``log_axes`` (loss, kick), the
    parameterisation of Section "Building histograms".  ``p_edges`` are the
    momentum-bin edges e_0 < ... < e_P in GeV/c.
    """

    p_edges: np.ndarray          # float64 [P+1]
    loss_lo: float
    loss_hi: float
    scat_lo: float
    scat_hi: float
    counts: np.ndarray           # uint32 [M][P][nL][nS]
    material_names: tuple = ()
    log_axes: tuple = (False, False)

    @property
    def n_mat(self) -> int:
        return int(self.counts.shape[0])

    @property
    def n_pbin(self) -> int:
        return int(self.counts.shape[1])

    @property
    def n_loss(self) -> int:
        return int(self.counts.shape[2])

    @property
    def n_scat(self) -> int:
        return int(self.counts.shape[3])


def log_edges(p_lo: float, p_hi: float, n_bins: int) -> np.ndarray:
    """Base-10 logarithmic momentum-bin edges p_lo * (p_hi/p_lo)^(i/n), i=0..n.

    The paper's validation binning is 95 such bins between 0.18 and 400 GeV
    (Section "Validation and benchmarking"; the binning itself is motivated in
    Section "Momentum binning").
    """
    i = np.arange(n_bins + 1, dtype=np.float64)
    e = 10.0 ** (math.log10(p_lo) + (math.log10(p_hi) - math.log10(p_lo)) * i / n_bins)
    e[0], e[-1] = p_lo, p_hi
    return e


def _moyal_cdf(v: np.ndarray, mu: float, sigma: float) -> np.ndarray:
    # f = mu + sigma * X with X = -ln Z^2, Z ~ N(0,1):  P(X <= x) = erfc(e^{-x/2}/sqrt 2)
    x = (v - mu) / sigma
    return special.erfc(np.exp(-0.5 * x) / math.sqrt(2.0))


def _rayleigh_cdf(v: np.ndarray, sigma: float) -> np.ndarray:
    return -np.expm1(-0.5 * (v / sigma) ** 2)


def _cell_probabilities(p_rep: float, a_m: float, x0: float, step: float,
                        l_edges: np.ndarray, s_edges: np.ndarray) -> np.ndarray:
    """Probability of each (loss, kick) cell for in-range, independent draws.

    Loss: Moyal with location mu = a_M d / p and scale 0.15 mu ("Landau-like").
    Kick: Rayleigh with scale equal to the Highland width
    0.0136/p * sqrt(d/X0) * (1 + 0.038 ln(d/X0)) ("Gaussian" in each
    transverse plane).  Draws outside the axis ranges are dropped, i.e. both
    distributions are truncated to the axes.
    """
    mu = a_m * step / p_rep
    sig_l = 0.15 * mu
    t = step / x0
    sig_s = 0.0136 / p_rep * math.sqrt(t) * (1.0 + 0.038 * math.log(t))
    cl = _moyal_cdf(l_edges, mu, sig_l)
    pl = np.diff(cl)
    if not np.isfinite(pl).all() or pl.sum() <= 0:
        # Whole loss mass outside the axis: keep it in the top cell.
        pl = np.zeros(len(l_edges) - 1)
        pl[-1 if mu > l_edges[-1] else 0] = 1.0
    cs = _rayleigh_cdf(s_edges, sig_s)
    ps = np.diff(cs)
    pl = np.clip(pl, 0.0, None) / np.clip(pl, 0.0, None).sum()
    ps = np.clip(ps, 0.0, None) / np.clip(ps, 0.0, None).sum()
    return np.outer(pl, ps).ravel()


def make_histograms(cfg_code: int, materials: tuple, p_edges: np.ndarray,
                    n_loss: int, n_scat: int, step: float,
                    loss_range=(0.0, 0.05), scat_range=(0.0, 5e-3),
                    n_fill: int = 1_000_000, log_axes=(False, False)) -> Histograms:
    """Fill one count histogram per (material, momentum bin).

    Each histogram holds exactly ``n_fill`` in-range (loss, kick) pairs drawn
    at the bin's representative momentum sqrt(e_i e_{i+1}).  Because loss and
    kick are independent, filling n_fill pairs into the 2D cells is the same
    as one multinomial draw over the product of the two binned marginals,
    which is what is done here (seeded per material and bin).
    """
    n_mat, n_pbin = len(materials), len(p_edges) - 1
    axis = lambda r, n, lg: np.geomspace(r[0], r[1], n + 1) if lg else np.linspace(r[0], r[1], n + 1)
    l_edges = axis(loss_range, n_loss, log_axes[0])
    s_edges = axis(scat_range, n_scat, log_axes[1])
    counts = np.empty((n_mat, n_pbin, n_loss, n_scat), dtype=np.uint32)
    for m, name in enumerate(materials):
        a_m, x0 = MATERIALS[name]
        for i in range(n_pbin):
            p_rep = math.sqrt(p_edges[i] * p_edges[i + 1])
            prob = _cell_probabilities(p_rep, a_m, x0, step, l_edges, s_edges)
            c = _rng(cfg_code, _PART_HIST, m, i).multinomial(n_fill, prob)
            counts[m, i] = c.reshape(n_loss, n_scat).astype(np.uint32)
    return Histograms(p_edges=np.asarray(p_edges, dtype=np.float64),
                      loss_lo=float(loss_range[0]), loss_hi=float(loss_range[1]),
                      scat_lo=float(scat_range[0]), scat_hi=float(scat_range[1]),
                      counts=counts, material_names=tuple(materials),
                      log_axes=(bool(log_axes[0]), bool(log_axes[1])))


def pilot_log_loss(material: str, p_probe: np.ndarray, step: float, k: int,
                   cfg_code: int) -> np.ndarray:
    """Pilot estimate of the mean log10 fractional loss at each probe momentum
    (the estimator of the appendix "Optimal Momentum Binning"): ``k`` draws of
    the loss recipe at each momentum, seeded per probe."""
    a_m, _ = MATERIALS[material]
    out = np.empty(len(p_probe))
    for j, p in enumerate(p_probe):
        mu = a_m * step / p
        z = _rng(cfg_code, _PART_HIST, 99, j).standard_normal(k)
        f = mu + 0.15 * mu * (-np.log(z * z))
        out[j] = np.mean(np.log10(f[f > 0]))
    return out


# --------------------------------------------------------------------------
# Geometry and field
# --------------------------------------------------------------------------
@dataclass
class Geometry:
    """Axis-aligned boxes; ``box[b] = (xlo, xhi, ylo, yhi, zlo, zhi)`` in m.

    Containment is half-open on every axis and overlapping boxes resolve to
    the lowest index.  ``material[b] = -1`` marks a vacuum box.  ``b_box[b]``
    is the uniform field of the box in tesla, multiplied by the field scale of
    magnet ``magnet[b]`` (``-1``: not scaled).  ``world = (x_max, y_max,
    z_max)`` are the break conditions |x| >= x_max, |y| >= y_max, z >= z_max.
    """

    box: np.ndarray              # float64 [n][6] ([0][6] when ``poly`` is given)
    material: np.ndarray         # int32 [n]
    b_box: np.ndarray            # float32 [n][3]
    magnet: np.ndarray           # int32 [n]
    n_mag: int
    world: np.ndarray            # float64 [3]
    # Convex blocks instead of boxes: [n][18] = z_lo, z_hi, the quadrilateral
    # at z_lo as (x, y) x 4, the one at z_hi (same vertex order).  The slice
    # at height z interpolates the two; containment is the sign test of the
    # edge cross products, half-open in z; lowest index wins.
    poly: Optional[np.ndarray] = None


@dataclass
class FieldMap:
    """Node-centred field samples on a regular grid (tesla).

    Node (i, j, k) sits at lo + (i, j, k) * (hi - lo) / (n - 1); ``b`` has
    shape [nz][ny][nx][3].  Outside [lo, hi] the map contributes zero.
    """

    lo: np.ndarray               # float64 [3]
    hi: np.ndarray               # float64 [3]
    b: np.ndarray                # float32 [nz][ny][nx][3]

    @property
    def shape_xyz(self):
        nz, ny, nx, _ = self.b.shape
        return nx, ny, nz


def _single_box(length: float, by: float) -> Geometry:
    return Geometry(
        box=np.array([[-1.0, 1.0, -1.0, 1.0, 0.0, length]], dtype=np.float64),
        material=np.array([0], dtype=np.int32),
        b_box=np.array([[0.0, by, 0.0]], dtype=np.float32),
        magnet=np.array([-1], dtype=np.int32),
        n_mag=0,
        world=np.array([1.0, 1.0, length], dtype=np.float64),
    )


def _slab_geometry(n_slab: int = 8, length: float = 5.0, by: float = 1.7) -> Geometry:
    dz = length / n_slab
    box = np.array([[-1.0, 1.0, -1.0, 1.0, m * dz, (m + 1) * dz] for m in range(n_slab)],
                   dtype=np.float64)
    box[-1, 5] = length
    return Geometry(box=box,
                    material=np.zeros(n_slab, dtype=np.int32),
                    b_box=np.tile(np.array([0.0, by, 0.0], dtype=np.float32), (n_slab, 1)),
                    magnet=np.arange(n_slab, dtype=np.int32),
                    n_mag=n_slab,
                    world=np.array([1.0, 1.0, length], dtype=np.float64))


# Shield stand-in: transverse layout of one station (x ranges, y ranges, material).
_IRON, _CONCRETE, _AIR = 0, 1, 2
_STATION_LAYOUT = (
    ((-1.2, -0.2), (-1.0, 1.0), _IRON),      # left yoke
    ((0.2, 1.2), (-1.0, 1.0), _IRON),        # right yoke
    ((-0.2, 0.2), (-1.0, 1.0), _AIR),        # air core
    ((-2.0, -1.2), (-2.0, 2.0), _CONCRETE),  # left wall
    ((1.2, 2.0), (-2.0, 2.0), _CONCRETE),    # right wall
)


def _shield(cfg_code: int):
    rng_g = _rng(cfg_code, _PART_GEOM)
    lengths = rng_g.uniform(2.0, 3.0, size=8)
    polarity = rng_g.choice([-1.0, 1.0], size=8)
    bmag = rng_g.uniform(1.5, 1.8, size=8)
    boxes, mats, magnets, zr = [], [], [], []
    z = 0.5
    for m in range(8):
        z0, z1 = z, z + lengths[m]
        zr.append((z0, z1))
        for b, ((x0, x1), (y0, y1), mat) in enumerate(_STATION_LAYOUT):
            boxes.append((x0, x1, y0, y1, z0, z1))
            mats.append(mat)
            magnets.append(m if b < 2 else -1)
        z = z1 + 0.5
    geom = Geometry(box=np.array(boxes, dtype=np.float64),
                    material=np.array(mats, dtype=np.int32),
                    b_box=np.zeros((len(boxes), 3), dtype=np.float32),
                    magnet=np.array(magnets, dtype=np.int32),
                    n_mag=8,
                    world=np.array([2.0, 2.0, 30.0], dtype=np.float64))
    # Field map: By = P_m B_m (+1 right yoke, -1 left yoke) times logistic
    # windows (5 cm wide) around each yoke, on 100 x 100 x 300 nodes.
    nx, ny, nz = 100, 100, 300
    lo = np.array([-2.0, -2.0, 0.0])
    hi = np.array([2.0, 2.0, 30.0])
    xs = np.linspace(lo[0], hi[0], nx)
    ys = np.linspace(lo[1], hi[1], ny)
    zs = np.linspace(lo[2], hi[2], nz)

    def win(u, a, b, w=0.05):
        return special.expit((u - a) / w) * special.expit((b - u) / w)

    wx_r = win(xs, 0.2, 1.2)
    wx_l = win(xs, -1.2, -0.2)
    wy = win(ys, -1.0, 1.0)
    by = np.zeros((nz, ny, nx), dtype=np.float64)
    for m, (z0, z1) in enumerate(zr):
        wz = win(zs, z0, z1)
        amp = polarity[m] * bmag[m]
        by += amp * wz[:, None, None] * wy[None, :, None] * (wx_r - wx_l)[None, None, :]
    b = np.zeros((nz, ny, nx, 3), dtype=np.float32)
    b[..., 1] = by.astype(np.float32)
    return geom, FieldMap(lo=lo, hi=hi, b=b)


def _quad(x0, x1, y0, y1):
    """Rectangle as a counter-clockwise quadrilateral [(x, y)] x 4."""
    return [x0, y0, x1, y0, x1, y1, x0, y1]


def _blocks(cfg_code: int) -> Geometry:
    """The shield stations as convex blocks: at the exit of station m the air
    core narrows by 2 s_m in x and the yokes follow it inwards and shrink by
    s_m / 2 in y (s_m ~ U(0, 0.15) m); the concrete walls stay prisms.  Yoke
    fields are uniform, (0, +-P_m B_m, 0) T, scaled by magnet m."""
    rng_g = _rng(cfg_code, _PART_GEOM)
    lengths = rng_g.uniform(2.0, 3.0, size=8)
    polarity = rng_g.choice([-1.0, 1.0], size=8)
    bmag = rng_g.uniform(1.5, 1.8, size=8)
    taper = rng_g.uniform(0.0, 0.15, size=8)
    blocks, mats, magnets, fields = [], [], [], []
    z = 0.5
    for m in range(8):
        z0, z1, s = z, z + lengths[m], taper[m]
        b = polarity[m] * bmag[m]
        layout = (
            (_quad(-1.2, -0.2, -1.0, 1.0), _quad(-1.2, -0.2 + s, -1.0 + s / 2, 1.0 - s / 2),
             _IRON, m, -b),
            (_quad(0.2, 1.2, -1.0, 1.0), _quad(0.2 - s, 1.2, -1.0 + s / 2, 1.0 - s / 2),
             _IRON, m, b),
            (_quad(-0.2, 0.2, -1.0, 1.0), _quad(-0.2 + s, 0.2 - s, -1.0, 1.0), _AIR, -1, 0.0),
            (_quad(-2.0, -1.2, -2.0, 2.0), _quad(-2.0, -1.2, -2.0, 2.0), _CONCRETE, -1, 0.0),
            (_quad(1.2, 2.0, -2.0, 2.0), _quad(1.2, 2.0, -2.0, 2.0), _CONCRETE, -1, 0.0),
        )
        for bottom, top, mat, mag, by in layout:
            blocks.append([z0, z1] + bottom + top)
            mats.append(mat)
            magnets.append(mag)
            fields.append((0.0, by, 0.0))
        z = z1 + 0.5
    n = len(blocks)
    return Geometry(box=np.zeros((0, 6)), material=np.array(mats, dtype=np.int32),
                    b_box=np.array(fields, dtype=np.float32),
                    magnet=np.array(magnets, dtype=np.int32), n_mag=8,
                    world=np.array([2.0, 2.0, 30.0], dtype=np.float64),
                    poly=np.array(blocks, dtype=np.float64).reshape(n, 18))


# --------------------------------------------------------------------------
# Muons
# --------------------------------------------------------------------------
@dataclass
class Muons:
    """Structure-of-arrays muon states: position (m), momentum (GeV/c), charge."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    px: np.ndarray
    py: np.ndarray
    pz: np.ndarray
    q: np.ndarray                # int8, +1 / -1

    def __len__(self) -> int:
        return int(self.x.shape[0])

    def take(self, idx) -> "Muons":
        return Muons(*(getattr(self, k)[idx] for k in ("x", "y", "z", "px", "py", "pz", "q")))

    def stacked(self) -> np.ndarray:
        """[6][n] float64 (x, y, z, px, py, pz)."""
        return np.stack([self.x, self.y, self.z, self.px, self.py, self.pz])


def _tiny_muons(n: int) -> Muons:
    j = np.arange(n)
    return Muons(x=np.zeros(n), y=np.zeros(n), z=np.full(n, -0.01),
                 px=np.zeros(n), py=np.zeros(n), pz=np.full(n, 100.0),
                 q=np.where(j % 2 == 0, 1, -1).astype(np.int8))


def _power_law_muons(cfg_code: int, n: int, z0: float) -> Muons:
    """C2 recipe: p ~ p^-2.7 on [10, 350] GeV, (x, y) ~ U(-0.5, 0.5) m,
    slopes ~ N(0, 10 mrad) in x and y, uniform charge."""
    g = lambda a: _rng(cfg_code, _PART_MUONS, a)
    u = g(0).random(n)
    a, b = 10.0 ** -1.7, 350.0 ** -1.7
    p = (a + u * (b - a)) ** (-1.0 / 1.7)
    q = np.where(g(1).random(n) < 0.5, 1, -1).astype(np.int8)
    x = g(2).uniform(-0.5, 0.5, n)
    y = g(3).uniform(-0.5, 0.5, n)
    tx = np.tan(g(4).normal(0.0, 0.010, n))
    ty = np.tan(g(5).normal(0.0, 0.010, n))
    norm = np.sqrt(tx * tx + ty * ty + 1.0)
    return Muons(x=x, y=y, z=np.full(n, z0), px=p * tx / norm, py=p * ty / norm,
                 pz=p / norm, q=q)


# --------------------------------------------------------------------------
# Whole workloads
# --------------------------------------------------------------------------
@dataclass
class RunParams:
    step: float                  # fixed step length d [m]
    max_steps: int
    p_min: float                 # GeV/c
    seed: int                    # Philox key
    n_variants: int = 1
    scales: Optional[np.ndarray] = None   # float32 [n_variants][n_mag] or None (= 1)
    sampler: int = 0             # 0 inverse CDF, 1 alias method
    interp: int = 0              # field map lookup: 0 trilinear, 1 nearest node
    stage_field: int = 0         # 0 field held from the step start, 1 at every RK4 stage


@dataclass
class Workload:
    name: str
    hist: Histograms
    geom: Geometry
    field: Optional[FieldMap]
    muons: Muons
    run: RunParams
    extra: dict = field(default_factory=dict)

    @property
    def n_lanes(self) -> int:
        return len(self.muons) * self.run.n_variants


DEFAULT_MUONS = {"tiny": 10_000, "block": 1_000_000, "shield": 10_000_000,
                 "scan": 1 << 17, "diff": 1_000_000, "blocks": 1_000_000,
                 "logbins": 1_000_000}

# Muons of the block-type workloads start a little before the first face; a
# start at -0.0075 m keeps step starts off the faces at multiples of 0.625 m
# (slabs) and at 0 and 5 m.
_Z0_BLOCK = -0.0075


def make_workload(name: str, n_muons: Optional[int] = None, n_fill: int = 1_000_000,
                  n_variants: Optional[int] = None) -> Workload:
    """Build one of the five seeded workloads (see the module docstring).

    ``n_muons`` truncates the muon list (exact prefix of the full list);
    ``n_fill`` sets the per-histogram fill count; ``n_variants`` (scan only)
    truncates the variant list.
    """
    if name not in CONFIGS:
        raise ValueError(f"unknown workload {name!r}; choose from {CONFIGS}")
    n = DEFAULT_MUONS[name] if n_muons is None else int(n_muons)
    step = 0.02
    if name == "tiny":
        edges = log_edges(1.0, 400.0, 32)
        hist = make_histograms(1, ("iron",), edges, 64, 64, step, n_fill=n_fill)
        geom = _single_box(1.0, 0.0)
        return Workload(name, hist, geom, None, _tiny_muons(n),
                        RunParams(step=step, max_steps=1000, p_min=1.0, seed=0))
    edges = log_edges(0.18, 400.0, 95)
    if name == "shield":
        hist = make_histograms(3, ("iron", "concrete", "air"), edges, 100, 100, step,
                               n_fill=n_fill)
        geom, fmap = _shield(3)
        return Workload(name, hist, geom, fmap, _power_law_muons(3, n, _Z0_BLOCK),
                        RunParams(step=step, max_steps=2000, p_min=0.18, seed=0))
    if name == "blocks":
        # the shield's histograms (seeded as workload 3), blocks seeded as 6
        hist = make_histograms(3, ("iron", "concrete", "air"), edges, 100, 100, step,
                               n_fill=n_fill)
        return Workload(name, hist, _blocks(6), None, _power_law_muons(6, n, _Z0_BLOCK),
                        RunParams(step=step, max_steps=2000, p_min=0.18, seed=0))
    if name == "logbins":
        hist = make_histograms(7, ("iron",), edges, 100, 100, step, loss_range=(1e-6, 1.0),
                               scat_range=(1e-6, 0.5), n_fill=n_fill, log_axes=(True, True))
        return Workload(name, hist, _single_box(5.0, 1.7), None,
                        _power_law_muons(2, n, _Z0_BLOCK),
                        RunParams(step=step, max_steps=1000, p_min=0.18, seed=0))
    # block, scan, diff share the block histograms (seeded as workload 2).
    hist = make_histograms(2, ("iron",), edges, 100, 100, step, n_fill=n_fill)
    if name == "block":
        return Workload(name, hist, _single_box(5.0, 1.7), None,
                        _power_law_muons(2, n, _Z0_BLOCK),
                        RunParams(step=step, max_steps=1000, p_min=0.18, seed=0))
    geom = _slab_geometry()
    if name == "scan":
        v = 64 if n_variants is None else int(n_variants)
        scales = _rng(4, _PART_VARIANTS).uniform(0.8, 1.2, size=(64, geom.n_mag))
        scales = scales[:v].astype(np.float32)
        return Workload(name, hist, geom, None, _power_law_muons(4, n, _Z0_BLOCK),
                        RunParams(step=step, max_steps=1000, p_min=0.18, seed=0,
                                  n_variants=v, scales=scales))
    # diff: unit scales, the block muons, transport to z = 5 m (<= 251 steps).
    return Workload(name, hist, geom, None, _power_law_muons(2, n, _Z0_BLOCK),
                    RunParams(step=step, max_steps=400, p_min=0.18, seed=0,
                              n_variants=1, scales=np.ones((1, geom.n_mag), np.float32)),
                    extra={"z_det": 30.0, "r_ap": 1.0, "r_scale": 0.01})
