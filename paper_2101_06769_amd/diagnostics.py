"""Host-side diagnostics of order-parameter fields (numpy, x fastest).

* Interface positions along a column: the phi = 1/2 crossings, linearly
  interpolated between the two cells that bracket them.  The Rayleigh-Taylor
  spike is the lowest crossing on the column through the perturbation trough
  and the bubble the highest crossing on the column through the crest
  (Sec. 3.2, 3.3).  Positions are reported in cells from the bottom wall, as
  multiples of the box width L as the paper plots them.
* Spreading radius of a drop impacting a liquid film (Sec. 3.4): the distance
  from the impact axis to the outermost point where the liquid (phi >= 1/2)
  reaches a sampling height just above the undisturbed film.  The paper
  compares it with r_K / D = 1.1 sqrt(t / T), T = D / U0.
"""
from __future__ import annotations

import numpy as np


def crossings(column, level=0.5):
    """Positions (in cell units, index space) where the 1-D profile crosses
    `level`, linearly interpolated, in increasing order."""
    c = np.asarray(column, dtype=np.float64) - level
    s = np.sign(c)
    idx = np.nonzero(s[:-1] * s[1:] < 0)[0]
    out = [i + c[i] / (c[i] - c[i + 1]) for i in idx]
    out += [float(i) for i in np.nonzero(c == 0)[0]]
    return sorted(out)


def rti_positions(phi, dim):
    """(spike, bubble) of a Rayleigh-Taylor run with heavy fluid on top and
    gravity along -y (2-D) or -z (3-D): the lowest phi = 1/2 crossing on the
    column through the trough of the initial cosine (x = L/2; (L/2, L/2) in
    3-D) and the highest crossing on the column through its crest (x = 0;
    (0, 0) in 3-D).  In cells from the bottom of the box; None where a column
    has no crossing."""
    phi = np.asarray(phi)
    if dim == 2:
        a = phi[0]                     # (ny, nx)
        nx = a.shape[1]
        trough, crest = a[:, nx // 2], a[:, 0]
    else:
        nz, ny, nx = phi.shape
        trough, crest = phi[:, ny // 2, nx // 2], phi[:, 0, 0]
    ct, cc = crossings(trough), crossings(crest)
    return (ct[0] if ct else None), (cc[-1] if cc else None)


def spreading_radius(phi, x_center, height, level=0.5):
    """Spreading radius of a 2-D impact: the largest |x - x_center| (in
    cells, linearly interpolated) at which phi >= level on the row at
    `height` (a fractional row index, interpolated between rows).  phi is
    (1, ny, nx) or (ny, nx)."""
    a = np.asarray(phi, dtype=np.float64)
    if a.ndim == 3:
        a = a[0]
    j = int(np.floor(height))
    f = height - j
    row = (1.0 - f) * a[j] + f * a[min(j + 1, a.shape[0] - 1)]
    xs = np.arange(row.size, dtype=np.float64)
    best = 0.0
    for xc in crossings(row, level):
        best = max(best, abs(xc - x_center))
    inside = row >= level
    if inside.any():
        best = max(best, float(np.abs(xs[inside] - x_center).max()))
    return best
