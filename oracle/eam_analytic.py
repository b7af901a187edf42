"""The paper's W EAM in closed form (oracle, FP64).

Appendix "AP potential for tungsten", subsections "EAM potential" and
"Optimising the EAM potential" (equations eam_F_Marinica, eam_Phi_Marinica,
eam_rho_Marinica, tungsten_rho_up, tungsten_F_up, tungsten_Phi_up and the
table of optimised parameters):

* embedding   xi^Fit(x) = a1 sqrt(x) + a2 x^2 + Delta xi;
* density     zeta_0(r) = sum_i a_i (d_i - r)^3 Theta(d_i - r), held at its
              value at r_cut below r_cut: zeta(r) = zeta_0(max(r, r_cut));
* pair        Phi(r) = sum_i a_i (d_i - r)^3 Theta(d_i - r) above r_hi, the
              quintic bridge sum_m b_m r^m on [r_lo, r_hi], and below r_lo the
              screened Coulomb (ZBL) energy Z1 Z2 / (4 pi eps0 r) phi(r / a)
              with phi(x) = sum_k c_k exp(-q_k x);
* energy      E_i = xi(sum_j zeta(r_ij)) + 1/2 sum_j Phi(r_ij)
              (section "EAM potential", equation for E_i^EAM).

Reading (the paper is silent there): the square root of the embedding is
undefined for x <= 0, so there xi = a2 x^2 + Delta xi (the x <= 0 branch
never occurs for an atom with a neighbour inside 4.9 A).  Theta(0) = 1 as
printed.
"""
from __future__ import annotations

import math

import numpy as np


class AnalyticWEam:
    def __init__(self, p):
        """p: dict with a_phi, d_phi, a_rho, d_rho, r_cut_rho, a_xi (2),
        d_xi, Z, eps0, a_zbl, zbl (pairs (c, q)), r_lo, r_hi, b_phi (6)."""
        self.p = p
        self.zeta_cut = self._knots(np.array([p["r_cut_rho"]]), p["a_rho"], p["d_rho"])[0][0]

    @staticmethod
    def _knots(r, a, d):
        r = np.asarray(r, dtype=np.float64)
        v = np.zeros_like(r)
        dv = np.zeros_like(r)
        for ai, di in zip(a, d):
            t = di - r
            on = t >= 0.0
            v = v + np.where(on, ai * t * t * t, 0.0)
            dv = dv + np.where(on, -3.0 * ai * t * t, 0.0)
        return v, dv

    def pair(self, r):
        p = self.p
        r = np.asarray(r, dtype=np.float64)
        pref = p["Z"] * p["Z"] / (4.0 * math.pi * p["eps0"])
        x = r / p["a_zbl"]
        phi = np.zeros_like(r)
        dphi = np.zeros_like(r)
        for c, q in p["zbl"]:
            e = np.exp(-q * x)
            phi = phi + c * e
            dphi = dphi - c * q / p["a_zbl"] * e
        zbl = pref * phi / r
        dzbl = pref * (dphi / r - phi / (r * r))
        b = p["b_phi"]
        poly = b[0] + r * (b[1] + r * (b[2] + r * (b[3] + r * (b[4] + r * b[5]))))
        dpoly = b[1] + r * (2 * b[2] + r * (3 * b[3] + r * (4 * b[4] + r * 5 * b[5])))
        knot, dknot = self._knots(r, p["a_phi"], p["d_phi"])
        v = np.where(r < p["r_lo"], zbl, np.where(r <= p["r_hi"], poly, knot))
        dv = np.where(r < p["r_lo"], dzbl, np.where(r <= p["r_hi"], dpoly, dknot))
        return v, dv

    def density(self, r):
        p = self.p
        r = np.asarray(r, dtype=np.float64)
        z, dz = self._knots(r, p["a_rho"], p["d_rho"])
        below = r <= p["r_cut_rho"]
        return np.where(below, self.zeta_cut, z), np.where(below, 0.0, dz)

    def embed(self, x):
        p = self.p
        x = np.asarray(x, dtype=np.float64)
        a1, a2 = p["a_xi"]
        pos = x > 0.0
        s = np.sqrt(np.where(pos, x, 1.0))
        v = np.where(pos, a1 * s, 0.0) + a2 * x * x + p["d_xi"]
        dv = np.where(pos, 0.5 * a1 / s, 0.0) + 2.0 * a2 * x
        return v, dv

    def energy_and_grad(self, d_list):
        """E_i^EAM, rho_i and dE_i/dd_ij for each atom's bond vectors."""
        n = len(d_list)
        E = np.zeros(n)
        rho = np.zeros(n)
        grads = []
        for i, d in enumerate(d_list):
            d = np.asarray(d, dtype=np.float64).reshape(-1, 3)
            r = np.sqrt(np.sum(d * d, -1))
            z, dz = self.density(r)
            ph, dph = self.pair(r)
            rho_i = float(np.sum(z))
            Fv, Fp = self.embed(np.array([rho_i]))
            E[i] = Fv[0] + 0.5 * float(np.sum(ph))
            rho[i] = rho_i
            grads.append(((Fp[0] * dz + 0.5 * dph) / r)[:, None] * d)
        return E, rho, grads
