"""FP64 velocity-Verlet (oracle; test infrastructure).

Kick-drift-kick with the paper's three groups (section "Nanoindentation":
a fixed bottom, a Nose-Hoover NVT layer above it and the NVE top): fixed
atoms keep their positions and zero velocity; positions are wrapped back into
the box in periodic dimensions (orthorhombic boxes); the indenter centre
moves with its constant velocity.  Units: A, fs, amu, eV; a = F/m * ACC.
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


KB = 8.617333262e-5          # eV / K


def layer_temperature(vel, masses, layer):
    """Kinetic temperature of the atoms in `layer`: 2K / (3 N k_B), with
    K = 1/2 sum m v^2 (m v^2 in amu A^2/fs^2 is converted to eV by 1/ACC)."""
    n = int(np.sum(layer))
    if n == 0:
        return 0.0
    v = vel[layer]
    two_k = float(np.sum(masses[layer][:, None] * v * v)) / ACC
    return two_k / (3.0 * n * KB)


def nh_half(vel, masses, layer, xi, eta, dt, T0, tau):
    """Half a step of the Nose-Hoover thermostat of the NVT region (section
    "Nanoindentation": the layer between the fixed bottom and the NVE top; its
    time constant tau is the step-4 entry of the equilibration table).

    Equations of motion of the layer: dv/dt = F/m - xi v,
    dxi/dt = (T / T0 - 1) / tau^2, deta/dt = xi.  Split symmetrically over
    dt/2: xi by dt/4 with the current T, eta by xi dt/2, v scaled by
    exp(-xi dt/2), xi by dt/4 with the scaled T.  Returns v, xi, eta."""
    xi = xi + 0.25 * dt * (layer_temperature(vel, masses, layer) / T0 - 1.0) / (tau * tau)
    eta = eta + 0.5 * dt * xi
    v = vel.copy()
    v[layer] = v[layer] * np.exp(-0.5 * dt * xi)
    xi = xi + 0.25 * dt * (layer_temperature(v, masses, layer) / T0 - 1.0) / (tau * tau)
    return v, xi, eta


def vv_step_nvt(pos, vel, forces, masses, fixed, layer, xi, eta, dt, T0, tau, box, periodic,
                force_fn, ind_centre=None, ind_vel=None):
    """Velocity-Verlet step with the Nose-Hoover layer: thermostat(dt/2),
    kick(dt/2), drift(dt), forces, kick(dt/2), thermostat(dt/2); the other
    mobile atoms are integrated at constant energy.
    Returns pos, vel, F, centre, xi, eta."""
    v, xi, eta = nh_half(vel, masses, layer, xi, eta, dt, T0, tau)
    x, v, F, c = vv_step(pos, v, forces, masses, fixed, dt, box, periodic, force_fn, ind_centre,
                         ind_vel)
    v, xi, eta = nh_half(v, masses, layer, xi, eta, dt, T0, tau)
    return x, v, F, c, xi, eta


def nh_extended_energy(kinetic, potential, n_layer, xi, eta, T0, tau):
    """Conserved quantity of the thermostatted dynamics:
    K + U + g k_B T0 (tau^2 xi^2 / 2 + eta) with g = 3 n_layer (the thermostat
    mass is Q = g k_B T0 tau^2)."""
    g = 3.0 * n_layer
    return kinetic + potential + g * KB * T0 * (0.5 * tau * tau * xi * xi + eta)


def kinetic_energy(vel, masses):
    return 0.5 * float(np.sum(masses[:, None] * vel * vel)) / ACC
