"""FP64 velocity-Verlet (oracle).

Kick-drift-kick with the paper's groups reduced to mobile and fixed atoms
(section "Nanoindentation": the bottom layers are kept fixed): fixed atoms
keep their positions and zero velocity; positions are wrapped back into the
box in periodic dimensions (orthorhombic boxes); the indenter centre moves
with its constant velocity.  Units: A, fs, amu, eV; a = F/m * ACC.
"""
from __future__ import annotations

import numpy as np

ACC = 9.648533212e-3


def wrap(pos, box, periodic):
    p = pos.copy()
    for k in range(3):
        if periodic[k]:
            L = box[k][k]
            x = p[:, k]
            p[:, k] = np.where(x >= L, x - L, np.where(x < 0.0, x + L, x))
    return p


def vv_step(pos, vel, forces, masses, fixed, dt, box, periodic, force_fn, ind_centre=None,
            ind_vel=None):
    """One step; force_fn(pos, ind_centre) -> forces.  Returns pos, vel, F, centre."""
    mob = (fixed == 0)[:, None]
    inv = (ACC / masses)[:, None]
    v = np.where(mob, vel + 0.5 * dt * forces * inv, 0.0)
    x = np.where(mob, pos + dt * v, pos)
    x = wrap(x, box, periodic)
    c = None
    if ind_centre is not None:
        c = np.asarray(ind_centre) + dt * np.asarray(ind_vel)
    F = force_fn(x, c)
    v = np.where(mob, v + 0.5 * dt * F * inv, 0.0)
    return x, v, F, c
