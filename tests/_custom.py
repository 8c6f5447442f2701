"""Small hand-built workloads for the oracle and parity pins."""
import numpy as np

from paper_2512_10520_amd import workloads as W


def flat_histograms(n_pbin=4, n_loss=8, n_scat=8, counts=None, p_lo=1.0, p_hi=1000.0,
                    loss=(0.0, 0.05), scat=(0.0, 5e-3), seed=7):
    """One material whose histograms are the same in every momentum bin."""
    if counts is None:
        rng = np.random.default_rng(seed)
        counts = rng.integers(0, 50, size=(n_loss, n_scat)).astype(np.uint32)
        counts[0, 0] = 0
        counts[n_loss - 1, n_scat - 1] += 1
    c = np.broadcast_to(counts, (1, n_pbin) + counts.shape).copy()
    return W.Histograms(p_edges=W.log_edges(p_lo, p_hi, n_pbin), loss_lo=loss[0],
                        loss_hi=loss[1], scat_lo=scat[0], scat_hi=scat[1], counts=c)


def geometry(boxes, materials, b_box=None, magnet=None, n_mag=0, world=(10.0, 10.0, 100.0),
             poly=None):
    """Boxes [n][6], or convex blocks ``poly`` [n][18] (then ``boxes`` is ignored)."""
    n = len(boxes) if poly is None else len(poly)
    return W.Geometry(box=np.zeros((0, 6)) if poly is not None
                      else np.asarray(boxes, np.float64).reshape(n, 6),
                      material=np.asarray(materials, np.int32).reshape(n),
                      b_box=np.zeros((n, 3), np.float32) if b_box is None
                      else np.asarray(b_box, np.float32).reshape(n, 3),
                      magnet=np.full(n, -1, np.int32) if magnet is None
                      else np.asarray(magnet, np.int32).reshape(n),
                      n_mag=n_mag, world=np.asarray(world, np.float64),
                      poly=None if poly is None else np.asarray(poly, np.float64).reshape(n, 18))


def muons(x, y, z, px, py, pz, q):
    b = np.broadcast_arrays(*(np.atleast_1d(np.asarray(v, np.float64)) for v in (x, y, z, px, py, pz)))
    n = b[0].shape[0]
    return W.Muons(*[np.ascontiguousarray(v) for v in b],
                   q=np.ascontiguousarray(np.broadcast_to(np.asarray(q, np.int8), (n,))))


def workload(hist, geom, mu, step=0.02, max_steps=1000, p_min=0.5, seed=0, field=None,
             scales=None, n_variants=1, sampler=0, interp=0, stage_field=0):
    return W.Workload("custom", hist, geom, field, mu,
                      W.RunParams(step=step, max_steps=max_steps, p_min=p_min, seed=seed,
                                  n_variants=n_variants, scales=scales, sampler=sampler,
                                  interp=interp, stage_field=stage_field))
