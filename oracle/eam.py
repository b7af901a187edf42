"""Embedded-atom method energy and bond gradients (oracle, FP64).

Paper, section "EAM potential", equation for E_i^EAM:
E_i = xi(sum_{j != i} zeta(r_ij)) + 1/2 sum_{j != i} Phi(r_ij)
with xi the embedding function, zeta the density and Phi the pair potential,
here given as tables (``tables``).  The gradient of E_i with respect to the
bond vector d_ij = r_j - r_i is [xi'(rho_i) zeta'(r) + Phi'(r)/2] d_ij/r.
"""
from __future__ import annotations

import numpy as np

from .tables import evaluate


def table_dict(t):
    return dict(x0=t.x0, dx=t.dx, n_knots=t.n_knots, coef=t.coef)


class EamOracle:
    def __init__(self, tables):
        self.phi = table_dict(tables.phi)
        self.rho = table_dict(tables.rho)
        self.F = table_dict(tables.F)

    def density(self, d):
        r = np.sqrt(np.sum(d * d, -1))
        return float(np.sum(evaluate(self.rho, r, "zero")[0]))

    def energy_and_grad(self, d_list):
        """E_i^EAM, rho_i and dE_i/dd_ij for each atom's bond vectors."""
        n = len(d_list)
        E = np.zeros(n)
        rho = np.zeros(n)
        grads = []
        for i, d in enumerate(d_list):
            d = np.asarray(d, dtype=np.float64).reshape(-1, 3)
            r = np.sqrt(np.sum(d * d, -1))
            z, dz = evaluate(self.rho, r, "zero")
            ph, dph = evaluate(self.phi, r, "zero")
            rho_i = float(np.sum(z))
            Fv, Fp = evaluate(self.F, np.array([rho_i]), "linear")
            E[i] = Fv[0] + 0.5 * float(np.sum(ph))
            rho[i] = rho_i
            grads.append(((Fp[0] * dz + 0.5 * dph) / r)[:, None] * d)
        return E, rho, grads
