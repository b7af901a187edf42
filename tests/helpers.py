"""Shared test helpers (test infrastructure; no method arithmetic)."""
import numpy as np

from oracle.ap import APOracle
from oracle.geometry import Systems


def total_energy(orc: APOracle, pos, box, periodic, lam, cutoff=5.5, sys_offset=None):
    n = len(pos)
    off = [0, n] if sys_offset is None else sys_offset
    S = Systems(pos, box, off, periodic, cutoff)
    return float(np.sum(orc.evaluate(S, lam)["e_atom"]))


def fd_forces(energy, pos, atoms, h=1e-4):
    """Central differences with one Richardson step, -dE/dr for selected atoms."""
    out = np.zeros((len(atoms), 3))
    for t, i in enumerate(atoms):
        for k in range(3):
            def d(hh):
                p = pos.copy(); p[i, k] += hh
                m = pos.copy(); m[i, k] -= hh
                return (energy(p) - energy(m)) / (2 * hh)
            out[t, k] = -(4 * d(h / 2) - d(h)) / 3
    return out


def jittered_bcc(n, a, sigma, seed):
    from paper_2505_12958_amd.workloads import lattice_points
    L = n * a
    p = lattice_points("bcc", (n, n, n), a)
    p = np.mod(p + np.random.default_rng(seed).normal(0, sigma, p.shape), L)
    return p, np.diag([L, L, L])[None].astype(np.float64)
