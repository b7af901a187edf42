"""Uniform-knot piecewise-cubic tables (oracle, FP64).

A table with knots x_k = x0 + k*dx (k = 0..n-1) stores, per interval k, the
cubic c0 + c1 t + c2 t^2 + c3 t^3 in t = x - x_k.  Evaluation rule:
k = clamp(floor((x - x0)/dx), 0, n-2); below x0 the first cubic is used.
Beyond the last knot a table is either zero ('zero', for Phi and zeta, whose
last knot is the cutoff) or the linear continuation of the last cubic with
its end slope ('linear', for the embedding F).
"""
from __future__ import annotations

import numpy as np


def evaluate(table, x, beyond="zero"):
    """Value and derivative of a table (dict with x0, dx, n_knots, coef)."""
    x = np.asarray(x, dtype=np.float64)
    x0, dx, n = float(table["x0"]), float(table["dx"]), int(table["n_knots"])
    coef = np.asarray(table["coef"], dtype=np.float64)
    k = np.floor((x - x0) / dx).astype(np.int64)
    k = np.clip(k, 0, n - 2)
    t = x - (x0 + k * dx)
    c0, c1, c2, c3 = coef[k, 0], coef[k, 1], coef[k, 2], coef[k, 3]
    v = c0 + t * (c1 + t * (c2 + t * c3))
    dv = c1 + t * (2.0 * c2 + t * 3.0 * c3)
    x_end = x0 + (n - 1) * dx
    past = x > x_end
    if np.any(past):
        ce = coef[n - 2]
        ve = ce[0] + dx * (ce[1] + dx * (ce[2] + dx * ce[3]))
        de = ce[1] + dx * (2.0 * ce[2] + dx * 3.0 * ce[3])
        if beyond == "zero":
            v = np.where(past, 0.0, v)
            dv = np.where(past, 0.0, dv)
        else:
            v = np.where(past, ve + de * (x - x_end), v)
            dv = np.where(past, de, dv)
    return v, dv
