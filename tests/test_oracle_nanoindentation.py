"""Pins of the nanoindentation protocol's oracle (section "Nanoindentation"
and the Results subsections: the Nose-Hoover NVT layer, the load P_ind, the
Hertz fit, the contact radius and the hardness) against what does not depend
on it: the thermostat's equations of motion solved by a general ODE
integrator, the conservation of its extended energy under real forces, the
Hertz theory's own contact radius, the geometry of a sphere cut by a plane,
and exact synthetic load curves."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import indentation as ind
from oracle import md
from oracle.ap import APOracle
from oracle.eam_analytic import AnalyticWEam
from oracle.geometry import Systems
from paper_2505_12958_amd import workloads as w
from paper_2505_12958_amd.workloads import lattice_points


def test_thermostat_of_free_atoms_follows_the_nose_hoover_equations():
    """Without forces the layer's 2K and xi obey d(2K)/dt = -2 xi 2K,
    dxi/dt = (T/T0 - 1)/tau^2, deta/dt = xi; the split integrator tracks the
    ODE solution to second order in dt/tau."""
    rng = np.random.default_rng(5)
    n = 40
    masses = np.full(n, w.MASS_W)
    vel = rng.normal(0.0, 0.0017, (n, 3))                 # about 600 K for W
    layer = np.ones(n, bool)
    layer[:8] = False                                     # NVE atoms: untouched by the thermostat
    T0, tau, dt, steps = 300.0, 40.0, 1.0, 300
    g = 3.0 * layer.sum()
    twok0 = float(np.sum(masses[layer, None] * vel[layer] ** 2)) / md.ACC

    def rhs(t, y):
        twok, xi, eta = y
        T = twok / (g * md.KB)
        return [-2.0 * xi * twok, (T / T0 - 1.0) / tau ** 2, xi]

    ts = dt * np.arange(1, steps + 1)
    ode = solve_ivp(rhs, (0.0, ts[-1]), [twok0, 0.0, 0.0], t_eval=ts, method="DOP853", rtol=1e-12,
                    atol=1e-14)
    x = np.zeros((n, 3))
    box = np.eye(3) * 1e4
    v, xi, eta = vel.copy(), 0.0, 0.0
    zero = lambda p, c: np.zeros_like(p)
    F = np.zeros((n, 3))
    Ts, xis, etas = [], [], []
    for _ in range(steps):
        x, v, F, _, xi, eta = md.vv_step_nvt(x, v, F, masses, np.zeros(n, np.uint8), layer, xi, eta, dt,
                                             T0, tau, box, (False,) * 3, zero)
        Ts.append(md.layer_temperature(v, masses, layer))
        xis.append(xi)
        etas.append(eta)
    T_ode = ode.y[0] / (g * md.KB)
    assert T_ode[0] > 1.5 * T0 or T_ode[0] < 0.7 * T0     # far from equilibrium: xi swings
    assert np.abs(np.array(Ts) - T_ode).max() < 2e-3 * T_ode.max()
    assert np.abs(np.array(xis) - ode.y[1]).max() < 2e-3 * np.abs(ode.y[1]).max()
    assert np.abs(np.array(etas) - ode.y[2]).max() < 2e-3 * np.abs(ode.y[2]).max()
    np.testing.assert_array_equal(v[~layer], vel[~layer])


def test_extended_energy_is_conserved_with_the_w_eam():
    """W crystal under the closed-form W EAM with the bottom half
    thermostatted from twice the target temperature: K + U drifts by the heat
    the thermostat removes while K + U + g k_B T0 (tau^2 xi^2/2 + eta) stays
    constant up to the integrator's O(dt^2) fluctuation."""
    weam = AnalyticWEam(dict(w.W_EAM, zbl=w.ZBL_C))
    orc = APOracle(eam_model=weam)
    nc = 3
    a = 3.165
    pos = lattice_points("bcc", (nc, nc, nc), a)
    n = len(pos)
    L = nc * a
    box = np.diag([L, L, L])
    per = (True, True, True)
    masses = np.full(n, w.MASS_W)
    rng = np.random.default_rng(11)
    vel = w.maxwell(rng, masses, np.ones(n, bool), 600.0)
    layer = pos[:, 2] < L / 2
    T0, tau, dt = 300.0, 25.0, 1.0
    lam = np.zeros(n)

    def evaluate(x):
        return orc.evaluate(Systems(x, box[None], [0, n], per, 5.5), lam)

    r = evaluate(pos)
    F, U = r["forces"], float(r["e_sys"][0])
    last = {}

    def force_fn(p, c):
        out = evaluate(p)
        last["U"] = float(out["e_sys"][0])
        return out["forces"]

    def run(layer):
        x, v, F2, xi, eta = pos.copy(), vel.copy(), F.copy(), 0.0, 0.0
        H0 = md.nh_extended_energy(md.kinetic_energy(v, masses), U, layer.sum(), xi, eta, T0, tau)
        E0 = md.kinetic_energy(v, masses) + U
        dH, dE = [], []
        for _ in range(120):
            x, v, F2, _, xi, eta = md.vv_step_nvt(x, v, F2, masses, np.zeros(n, np.uint8), layer, xi, eta,
                                                  dt, T0, tau, box, per, force_fn)
            K = md.kinetic_energy(v, masses)
            dH.append(md.nh_extended_energy(K, last["U"], layer.sum(), xi, eta, T0, tau) - H0)
            dE.append(K + last["U"] - E0)
        return np.abs(np.array(dH)), np.abs(np.array(dE))

    dH, dE = run(layer)
    _, dE_nve = run(np.zeros(n, bool))                     # no thermostat: velocity Verlet's own fluctuation
    assert dE.max() > 0.5                                  # the thermostat removed real heat (eV)
    assert dE.max() > 30.0 * dE_nve.max()
    assert dH.max() < 1.5 * dE_nve.max()


def test_hertz_load_matches_the_hertz_contact_radius():
    """Hertz theory for a rigid sphere on an elastic half-space: the contact
    radius a = (3 P R / (4 E*))^(1/3) and the depth h = a^2 / R; the load
    formula must reproduce both."""
    R, E = 60.0, 3.2
    h = np.linspace(0.1, 8.0, 30)
    P = ind.hertz_load(h, E, R)
    a = (3.0 * P * R / (4.0 * E)) ** (1.0 / 3.0)
    np.testing.assert_allclose(a * a / R, h, rtol=1e-13)
    assert np.all(ind.hertz_load(np.array([-1.0, 0.0]), E, R) == 0.0)


def test_contact_radius_is_the_chord_of_the_sphere_at_the_surface():
    """The sphere of radius R whose lowest point is h below the plane cuts the
    plane in a circle; its radius found by bisection on |p - c| = R."""
    R = 60.0
    for h in (0.5, 4.0, 20.8, 60.0, 100.0):
        lo, hi = 0.0, R
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if math.hypot(mid, R - h) < R:
                lo = mid
            else:
                hi = mid
        assert abs(float(ind.contact_radius(h, R)) - lo) < 1e-9
    assert float(ind.contact_radius(-2.0, R)) == 0.0


def test_hertz_fit_recovers_the_modulus_and_ignores_points_outside_the_range():
    R = 60.0
    E = 519.0 / ind.EV_A3_TO_GPA                           # the paper's EAM value for W, eV/A^3
    h = np.linspace(-4.2, 12.0, 400)
    P = ind.hertz_load(h, E, R)
    P_plastic = np.where(h > 8.3, 0.6 * P, P)             # a load drop past the elastic limit
    assert abs(ind.hertz_fit(h, P_plastic, R, 8.3) - E) < 1e-12 * E
    rng = np.random.default_rng(2)
    noisy = P + rng.normal(0.0, 0.5, P.shape)
    assert abs(ind.hertz_fit(h, noisy, R, 8.3) - E) < 0.02 * E
    with pytest.raises(ValueError):
        ind.hertz_fit(h, P, R, -5.0)


def test_depth_and_hardness():
    R, zs = 60.0, 100.0
    assert float(ind.depth(zs + R + 4.2, R, zs)) == pytest.approx(-4.2, abs=1e-12)
    assert float(ind.depth(zs + R - 3.0, R, zs)) == pytest.approx(3.0, abs=1e-12)
    h = np.array([-1.0, 2.0, 10.0])
    P = np.array([0.0, 50.0, 900.0])
    pm = ind.mean_contact_pressure(P, h, R)
    assert math.isnan(pm[0])
    np.testing.assert_allclose(pm[1:], P[1:] / (math.pi * h[1:] * (2 * R - h[1:])), rtol=1e-14)
