"""Host-side FP64 observables of the wetting campaigns (validation, not the step).

- contact_patch_radius: radius of the contact area of a droplet mesh on a
  wall plane, the r of the spreading law (Eq. tanner_law);
- power_law_fit: C and delta of r/R = C (t/t*)^delta over the spreading
  window of a sampled r(t).
"""
from __future__ import annotations

import math

import numpy as np


def contact_patch_radius(q: np.ndarray, faces: np.ndarray, z_wall: float = 0.5, band: float = 1.0,
                         wall: int = 0) -> float:
    """Equivalent radius sqrt(A / pi) of the contact area A: the area,
    projected on the wall plane, of the faces whose three vertices all lie
    within `band` of the plane z = z_wall (wall 0: the plane below the
    droplet, heights z - z_wall; 1: above it, heights z_wall - z).
    q: [nv, 3], faces: [nf, 3]."""
    q = np.asarray(q, dtype=np.float64)
    faces = np.asarray(faces)
    h = q[:, 2] - z_wall if wall == 0 else z_wall - q[:, 2]
    near = h < band
    sel = faces[near[faces].all(axis=1)]
    if len(sel) == 0:
        return 0.0
    a, b, c = q[sel[:, 0]], q[sel[:, 1]], q[sel[:, 2]]
    area = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    return math.sqrt(area.sum() / math.pi)


def power_law_fit(t: np.ndarray, r: np.ndarray, R: float, t_star: float, x_min: float = 0.2,
                  frac: float = 0.9) -> dict:
    """Least-squares fit of log(r/R) = log C + delta log(t/t*) over the
    spreading window: the samples with t/t* >= x_min, r > 0, up to the first
    sample where r reaches `frac` of its largest value (the approach to the
    plateau, where the power law ends, is left out).  Returns delta, C, the
    window in t/t* and the number of samples used."""
    t = np.asarray(t, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    x, y = t / t_star, r / R
    stop = np.argmax(r >= frac * r.max())
    keep = (x >= x_min) & (y > 0) & (np.arange(len(t)) <= stop)
    if keep.sum() < 3:
        raise ValueError("fewer than 3 samples in the spreading window")
    lx, ly = np.log(x[keep]), np.log(y[keep])
    A = np.stack([np.ones_like(lx), lx], axis=1)
    (lc, delta), *_ = np.linalg.lstsq(A, ly, rcond=None)
    return {"delta": float(delta), "C": float(math.exp(lc)), "window_t_over_tstar": [float(x[keep][0]),
                                                                                     float(x[keep][-1])],
            "samples": int(keep.sum())}
