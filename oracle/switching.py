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


def lambda_and_gradient(pos, rule):
    """lambda_i and d lambda_i / d r_i of a geometric rule (sphere,
    hemisphere, mask): nonzero only in the cosine band r_full < d < r_full +
    taper, and zero where the mask or the surface override fixes lambda.
    Constant and given rules have no gradient."""
    pos = np.asarray(pos, dtype=np.float64)
    lam = lambda_of(pos, rule)
    grad = np.zeros_like(pos)
    if rule.kind in (1, 2, 3):
        dvec = pos - np.asarray(rule.centre)[None, :]
        d = np.sqrt(np.sum(dvec * dvec, axis=1))
        band = (d > rule.r_full) & (d < rule.r_full + rule.taper)
        fixed = np.zeros(len(pos), bool)
        if rule.kind == 3 and rule.mask is not None:
            fixed |= np.asarray(rule.mask) != 0
        band &= ~fixed
        dl = -0.5 * math.pi / rule.taper * np.sin(math.pi * (d - rule.r_full) / rule.taper)
        grad[band] = (dl[band] / d[band])[:, None] * dvec[band]
    return lam, grad


def ace_list(lam):
    """Indices with lambda > 0, ascending."""
    return np.nonzero(np.asarray(lam) > 0.0)[0]


# ---------------------------------------------------------------------------
# Dynamic switching (section "Adaptive-precision potential" and the appendix
# "Switching function" with the table of the adaptive-precision model's
# parameters).  The paper takes the detection from the centro-symmetry
# parameter (CSP) of the 14 nearest neighbours, averaged over time, maps it
# to the switching parameter between CSP_lo and CSP_hi, spreads the precise
# region by a spatial transition zone between r_lo and r_hi, averages the
# result over time, snaps values within dlambda_min of 0 or 1, and fixes the
# detection value in two zones (a precise hemisphere under the tip, fast
# surface atoms outside it).  The formulas themselves belong to the cited
# adaptive-precision method, which is not part of the paper; the readings
# taken here (all in the ACE-weight convention mu = 1 - lambda_paper):
#
#   CSP_i   = sum of the n/2 smallest |d_a + d_b|^2 over the pairs a < b of
#             the n nearest neighbours (n = 14; ranked by the canonical r^2,
#             ties by index); r^2 and the pair sums in FP64 with every
#             operation rounded separately, the n/2 values summed in
#             ascending order; an atom with fewer than n neighbours within
#             the cutoff r_c gets the largest value a full set could have,
#             (n/2) (2 r_c)^2 (always detected, finite for the averages);
#   average c_i <- c_i + (CSP_i - c_i) / N_csp (the first update sets c_i);
#   mu0_i   = 0 for c_i <= CSP_lo, 1 for c_i >= CSP_hi, between
#             (1 - cos(pi (c_i - CSP_lo)/(CSP_hi - CSP_lo)))/2;
#             mu0_i = 1 inside the precise ball (|r_i - centre|^2 <=
#             r_precise^2, the squared distance summed as (x^2 + y^2) + z^2),
#             else mu0_i = 0 for surface atoms (z_i >= z_surface_min);
#   mu_i    = max over j (including i) with r_ij^2 < r_hi^2 of mu0_j g(r_ij),
#             g = 1 for r <= r_lo, (1 + cos(pi (r - r_lo)/(r_hi - r_lo)))/2
#             below r_hi (canonical minimum-image displacement r_i - r_j);
#   average m_i <- m_i + (mu_i - m_i) / N_lambda (the first update sets m_i);
#   lambda_i = 0 if m_i < dlambda_min, 1 if m_i > 1 - dlambda_min, else m_i.
#
# Parity unpinned: the time averaging, the ramp and transition shapes and
# the snapping are readings of the absent method paper; the pins below fix
# the CSP definition, the closed forms of each step and their composition.

from dataclasses import dataclass

from .geometry import displacement, r2_of


@dataclass
class SwitchParams:
    csp_lo: float = 1.5
    csp_hi: float = 1.6
    n_csp: int = 14
    n_csp_avg: int = 110
    r_lo: float = 4.0
    r_hi: float = 12.0
    n_lambda_avg: int = 110
    dlambda_min: float = 0.01
    centre: tuple = (0.0, 0.0, 0.0)
    r_precise: float = -1.0
    z_surface_min: float = float("inf")


def csp_of(d, n_nb=14, rc=5.5):
    """CSP of one atom from its bond vectors d[j, 3] in neighbour-index order
    (ties in r^2 keep that order); rc: the neighbour-list cutoff."""
    d = np.asarray(d, dtype=np.float64).reshape(-1, 3)
    if len(d) < n_nb:
        return (n_nb // 2) * (2.0 * rc) * (2.0 * rc)
    r2 = r2_of(d)
    near = d[np.argsort(r2, kind="stable")[:n_nb]]
    sums = []
    for a in range(n_nb):
        for b in range(a + 1, n_nb):
            s = near[a] + near[b]
            sums.append((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2])
    total = 0.0
    for v in sorted(sums)[: n_nb // 2]:
        total += v
    return total


def csp_all(S, rows, n_nb=14):
    """CSP of every atom; rows[i] = (j ascending, d) neighbour lists."""
    return np.array([csp_of(rows[i][1], n_nb, S.cutoff) for i in range(S.n_atoms)])


def ramp(c, lo, hi):
    c = np.asarray(c, dtype=np.float64)
    t = np.clip((c - lo) / (hi - lo), 0.0, 1.0)
    return np.where(c <= lo, 0.0, np.where(c >= hi, 1.0, 0.5 * (1.0 - np.cos(math.pi * t))))


def transition(r, r_lo, r_hi):
    r = np.asarray(r, dtype=np.float64)
    band = 0.5 * (1.0 + np.cos(math.pi * (r - r_lo) / (r_hi - r_lo)))
    return np.where(r <= r_lo, 1.0, np.where(r < r_hi, band, 0.0))


def detection(pos, c_avg, p: SwitchParams):
    mu0 = ramp(c_avg, p.csp_lo, p.csp_hi)
    if p.r_precise > 0:
        inside = r2_of(pos - np.asarray(p.centre)[None, :]) <= p.r_precise * p.r_precise
    else:
        inside = np.zeros(len(pos), bool)
    surf = (pos[:, 2] >= p.z_surface_min) & ~inside
    return np.where(inside, 1.0, np.where(surf, 0.0, mu0))


def spread(S, mu0, p: SwitchParams):
    """mu_i = max_j mu0_j g(r_ij) over sources j with mu0_j > 0 (brute force
    over every atom of the source's system, minimum image)."""
    mu = np.zeros(S.n_atoms)
    for j in np.nonzero(mu0 > 0)[0]:
        s = S.sys_of[j]
        lo, hi = S.sys_offset[s], S.sys_offset[s + 1]
        d = displacement(S.pos[j][None, :], S.pos[lo:hi], S.box[s], S.periodic, S.Hi[s])
        r2 = r2_of(d)
        g = np.where(r2 < p.r_hi * p.r_hi, transition(np.sqrt(r2), p.r_lo, p.r_hi), 0.0)
        mu[lo:hi] = np.maximum(mu[lo:hi], mu0[j] * g)
    return mu


def snap(m, dmin):
    m = np.asarray(m, dtype=np.float64)
    return np.where(m < dmin, 0.0, np.where(m > 1.0 - dmin, 1.0, m))


class DynamicSwitching:
    """State (time averages) and one update per call, in the order above."""

    def __init__(self, params: SwitchParams):
        self.p = params
        self.c_avg = None
        self.m_avg = None

    def update(self, S, rows=None):
        p = self.p
        rows = S.neighbour_lists() if rows is None else rows
        c = csp_all(S, rows, p.n_csp)
        self.c_avg = c.copy() if self.c_avg is None else self.c_avg + (c - self.c_avg) / p.n_csp_avg
        mu0 = detection(S.pos, self.c_avg, p)
        mu = spread(S, mu0, p)
        self.m_avg = mu.copy() if self.m_avg is None else self.m_avg + (mu - self.m_avg) / p.n_lambda_avg
        return snap(self.m_avg, p.dlambda_min)
