"""Analysis of a nanoindentation run (oracle, FP64; test infrastructure).

Section "Results" (Cu and W subsections), equations hertz_fit, p_m and
contact_radius:

* Hertzian load      P_H(h) = 4/3 E* R^(1/2) h^(3/2) for h > 0 (zero above
                     the surface);
* indentation modulus E* from the load curve P_ind(h) in the elastic range:
                     the one-parameter least-squares fit of P_H to P_ind over
                     the points with 0 < h <= h_fit;
* contact radius     a_c = sqrt(h (2R - h));
* hardness           p_m = P_ind / (pi a_c^2).

Readings (the paper does not state them): h is the depth of the indenter's
lowest point below the reference surface height z_surface, h = z_surface -
(z_centre - R), so the indenter starts at h_0 < 0; the fit range h_fit is the
caller's (the paper fits the elastic part before the first load drop).
Units: A, eV; E* and p_m come out in eV/A^3 (times EV_A3_TO_GPA for GPa).
"""
from __future__ import annotations

import math

import numpy as np

EV_A3_TO_GPA = 160.21766208


def depth(centre_z, R, z_surface):
    """Indentation depth of the tip's lowest point below z_surface."""
    return z_surface - (np.asarray(centre_z, dtype=np.float64) - R)


def hertz_load(h, E_star, R):
    h = np.asarray(h, dtype=np.float64)
    hp = np.where(h > 0.0, h, 0.0)
    return 4.0 / 3.0 * E_star * math.sqrt(R) * hp * np.sqrt(hp)


def hertz_fit(h, P, R, h_fit):
    """E* minimising sum (P_i - P_H(h_i))^2 over 0 < h_i <= h_fit: the
    normal equation of a model linear in E*, E* = sum P w / sum w^2 with
    w = 4/3 R^(1/2) h^(3/2)."""
    h = np.asarray(h, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    sel = (h > 0.0) & (h <= h_fit)
    if not np.any(sel):
        raise ValueError("no load points with 0 < h <= h_fit")
    w = 4.0 / 3.0 * math.sqrt(R) * h[sel] ** 1.5
    return float(np.sum(P[sel] * w) / np.sum(w * w))


def contact_radius(h, R):
    h = np.asarray(h, dtype=np.float64)
    return np.sqrt(np.clip(h * (2.0 * R - h), 0.0, None))


def mean_contact_pressure(P, h, R):
    """p_m = P / (pi a_c^2); NaN where a_c = 0 (no contact)."""
    a = contact_radius(h, R)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(a > 0.0, np.asarray(P, dtype=np.float64) / (math.pi * a * a), np.nan)
