"""Per-atom switching parameter lambda_i (oracle, FP64).

Paper, section "Adaptive-precision potential": E_i = lambda_i E_i^EAM +
(1 - lambda_i) E_i^ACE with the region under the indenter always precise and
surface atoms outside that region always fast.  Here lambda is the ACE
weight (lambda = 1 - lambda_paper).  Rules:

* const:      lambda = value;
* sphere / hemisphere: with d = |r - centre| (plain Euclidean distance),
  lambda = 1 for d <= r_full, (1 + cos(pi (d - r_full)/taper))/2 for
  r_full < d < r_full + taper, 0 beyond (the hemisphere's centre is the
  first-contact point on the surface; atoms of the solid below it fill the
  half-ball);
* mask:       the hemisphere rule, raised to 1 where mask_i = 1 (a
  centro-symmetry threshold computed once at set-up);
* for sphere/hemisphere/mask rules: atoms with z >= z_surface_min whose
  geometric lambda is 0 are forced to lambda = 0 (fast surface).
"""
from __future__ import annotations

import math

import numpy as np


def geometric(pos, centre, r_full, taper):
    d = np.sqrt(np.sum((pos - np.asarray(centre)[None, :]) ** 2, axis=1))
    lam = np.where(d <= r_full, 1.0, 0.0)
    band = (d > r_full) & (d < r_full + taper)
    lam = np.where(band, 0.5 * (1.0 + np.cos(math.pi * (d - r_full) / taper)), lam)
    return lam


def lambda_of(pos, rule):
    pos = np.asarray(pos, dtype=np.float64)
    if rule.kind == 0:
        return np.full(len(pos), float(rule.value))
    lam = geometric(pos, rule.centre, rule.r_full, rule.taper)
    geo_zero = lam == 0.0
    if rule.kind == 3 and rule.mask is not None:
        lam = np.where(np.asarray(rule.mask) != 0, 1.0, lam)
    surf = (pos[:, 2] >= rule.z_surface_min) & geo_zero
    return np.where(surf, 0.0, lam)


def ace_list(lam):
    """Indices with lambda > 0, ascending."""
    return np.nonzero(np.asarray(lam) > 0.0)[0]
