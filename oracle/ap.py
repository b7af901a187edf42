"""AP blend, forces at fixed lambda, virial, indenter (oracle, FP64).

Energy (paper, equation E_i of the AP potential, lambda = ACE weight):
    E = sum_i [lambda_i E_i^ACE + (1 - lambda_i) E_i^EAM] + E_ind.
lambda is a per-atom input held fixed during one evaluation, so the forces
are F = -dE/dr at fixed lambda:  with G_ij = d(w E_i)/d d_ij for each bond
(d_ij = r_j - r_i), F_i += G_ij and F_j -= G_ij.  Virial W = -sum_i sum_j
d_ij (x) G_ij (per system), which equals -dE/d(strain).

Indenter (paper, equation V_ind and the load equation): for every mobile atom
at distance delta = |r - r_ind| < R, V = K/3 (R - delta)^3 and
F = K (R - delta)^2 (r - r_ind)/delta; the load is the sum of the indenter
forces projected on the indentation direction.
"""
from __future__ import annotations

import numpy as np

from .ace import AceOracle
from .eam import EamOracle
from .geometry import Systems


def indenter(pos, mobile, centre, R, K, direction=(0.0, 0.0, -1.0)):
    """Energy, forces (N, 3) and load of the spherical indenter."""
    d = pos - np.asarray(centre)[None, :]
    delta = np.sqrt(np.sum(d * d, 1))
    inside = (delta < R) & mobile
    f = np.zeros_like(pos)
    pen = np.where(inside, R - delta, 0.0)
    E = float(np.sum(K / 3.0 * pen ** 3))
    f[inside] = (K * pen[inside] ** 2 / delta[inside])[:, None] * d[inside]
    load = float(np.sum(f @ np.asarray(direction)))
    return E, f, load


class APOracle:
    def __init__(self, eam_tables=None, ace_model=None, eam_model=None):
        """eam_model: an EAM object with energy_and_grad (e.g. the closed-form
        W EAM of eam_analytic) used instead of tables."""
        if eam_model is not None:
            self.eam = eam_model
        else:
            self.eam = EamOracle(eam_tables) if eam_tables is not None else None
        self.ace = AceOracle(ace_model) if ace_model is not None else None

    def bond_terms(self, sysm, lam, atoms, nl):
        """Per atom in `atoms`: unweighted E^EAM, E^ACE and weighted bond grads.

        nl: dict atom -> (j, d).  Returns e_eam, e_ace, G (list, sum of
        (1-lam) dE^EAM/dd and lam dE^ACE/dd), rho, phi."""
        n = len(atoms)
        e_eam = np.zeros(n)
        e_ace = np.zeros(n)
        rho = np.zeros(n)
        phi = np.zeros((n, 2))
        G = [np.zeros((len(nl[i][0]), 3)) for i in atoms]
        w = np.array([1.0 - lam[i] for i in atoms])
        if self.eam is not None:
            sel = [k for k in range(n) if w[k] > 0.0]
            if sel:
                E, r, g = self.eam.energy_and_grad([nl[atoms[k]][1] for k in sel])
                for t, k in enumerate(sel):
                    e_eam[k] = E[t]
                    rho[k] = r[t]
                    G[k] = G[k] + w[k] * g[t]
        if self.ace is not None:
            sel = [k for k in range(n) if lam[atoms[k]] > 0.0]
            if sel:
                E, g, ph, _ = self.ace.energy_and_grad([nl[atoms[k]][1] for k in sel])
                for t, k in enumerate(sel):
                    e_ace[k] = E[t]
                    phi[k] = ph[t]
                    G[k] = G[k] + lam[atoms[k]] * g[t]
        return e_eam, e_ace, G, rho, phi

    def evaluate(self, sysm: Systems, lam, nl=None, indenter_args=None, mobile=None,
                 lambda_rule=None):
        """Full evaluation: per-atom energies, forces, per-system energy and virial.

        lambda_rule (a geometric switching rule): lambda is the rule's value
        at these positions and the forces are the full -dE/dr with
        lambda = lambda(r): the fixed-lambda forces plus
        -(E_i^ACE - E_i^EAM) d lambda_i / d r_i on each atom of the taper
        band, whose virial is -(r_i - centre) (x) (E_i^ACE - E_i^EAM)
        d lambda_i / d r_i."""
        N = sysm.n_atoms
        lam = np.asarray(lam, dtype=np.float64)
        if nl is None:
            nl = sysm.neighbour_lists_fast() if N > 3000 else sysm.neighbour_lists()
        nld = {i: nl[i] for i in range(N)}
        atoms = list(range(N))
        e_eam, e_ace, G, rho, phi = self.bond_terms(sysm, lam, atoms, nld)
        e_atom = lam * e_ace + (1.0 - lam) * e_eam
        F = np.zeros((N, 3))
        ns = len(sysm.box)
        Wv = np.zeros((ns, 3, 3))
        for i in range(N):
            js, d = nl[i]
            if len(js) == 0:
                continue
            g = G[i]
            F[i] += g.sum(0)
            np.subtract.at(F, js, g)
            Wv[sysm.sys_of[i]] -= d.T @ g
        if lambda_rule is not None:
            from .switching import lambda_and_gradient
            lam_r, grad = lambda_and_gradient(sysm.pos, lambda_rule)
            if np.any(lam_r != lam):
                raise ValueError("lambda_rule does not give the lambda passed in")
            G = (e_ace - e_eam)[:, None] * grad
            F -= G
            dvec = sysm.pos - np.asarray(lambda_rule.centre)[None, :]
            for i in np.nonzero(np.any(G != 0.0, axis=1))[0]:
                Wv[sysm.sys_of[i]] -= np.outer(dvec[i], G[i])
        e_sys = np.array([e_atom[sysm.sys_offset[s]:sysm.sys_offset[s + 1]].sum() for s in range(ns)])
        out = dict(e_atom=e_atom, e_eam=e_eam, e_ace=e_ace, forces=F, virial=Wv, e_sys=e_sys,
                   rho=rho, phi=phi, nl=nl, lam=lam)
        if indenter_args is not None and indenter_args.get("K", 0.0) > 0.0:
            mob = np.ones(N, bool) if mobile is None else mobile
            Ei, Fi, load = indenter(sysm.pos, mob, indenter_args["centre"], indenter_args["R"],
                                    indenter_args["K"])
            out["forces"] = F + Fi
            out["e_ind"] = Ei
            out["load"] = load
        return out

    def forces_at(self, sysm: Systems, lam, atoms, finder=None):
        """Forces on selected atoms only, from the neighbour lists of those
        atoms and of their neighbours (for full-size sampled checks); finder
        defaults to the brute-force Systems.neighbours_of."""
        lam = np.asarray(lam, dtype=np.float64)
        nld = {}
        finder = sysm.neighbours_of if finder is None else finder

        def get(i):
            if i not in nld:
                nld[i] = finder(i)
            return nld[i]

        need = set()
        for k in atoms:
            js, _ = get(int(k))
            need.add(int(k))
            need.update(int(j) for j in js)
        need = sorted(need)
        for i in need:
            get(i)
        e_eam, e_ace, G, rho, phi = self.bond_terms(sysm, lam, need, nld)
        pos_of = {a: t for t, a in enumerate(need)}
        F = np.zeros((len(atoms), 3))
        for t, k in enumerate(atoms):
            k = int(k)
            js, _ = nld[k]
            F[t] += G[pos_of[k]].sum(0)
            for j in js:
                jl, _ = nld[int(j)]
                s = int(np.searchsorted(jl, k))
                F[t] -= G[pos_of[int(j)]][s]
        e = {a: (lam[a] * e_ace[pos_of[a]] + (1 - lam[a]) * e_eam[pos_of[a]]) for a in need}
        return F, np.array([e[int(k)] for k in atoms]), {a: nld[a] for a in atoms}
