"""Pins of the EAM oracle against the paper's W EAM (appendix, table of
optimised parameters, and the 'fit' column of the table of properties)."""
import json
import math
import os

import numpy as np
import pytest

from oracle.eam import EamOracle
from oracle.geometry import Systems
from oracle.tables import evaluate
from paper_2505_12958_amd import workloads as w
from paper_2505_12958_amd.workloads import lattice_points

EV_A3_TO_GPA = 160.21766208
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "w_eam_fit_properties.json")))


@pytest.fixture(scope="module")
def wtab():
    return EamOracle(w.make_eam_tables("W", noise=0.0))


def energy_per_atom(orc, a, eps=None, n=4):
    p = lattice_points("bcc", (n, n, n), a)
    H = np.eye(3) * n * a
    if eps is not None:
        F = np.eye(3) + eps
        p = p @ F.T
        H = H @ F.T
    S = Systems(p, H[None], [0, len(p)], (True, True, True), 5.5)
    nl = S.neighbour_lists()
    E, _, _ = orc.energy_and_grad([x[1] for x in nl])
    return E.sum() / len(p), abs(np.linalg.det(H)) / len(p)


def lattice_min(orc):
    lo, hi = 3.15, 3.22
    g = (math.sqrt(5) - 1) / 2
    for _ in range(60):
        x1, x2 = hi - g * (hi - lo), lo + g * (hi - lo)
        if energy_per_atom(orc, x1)[0] < energy_per_atom(orc, x2)[0]:
            hi = x2
        else:
            lo = x1
    return 0.5 * (lo + hi)


def test_w_eam_lattice_constant_and_cohesive_energy(wtab):
    a0 = lattice_min(wtab)
    e0, _ = energy_per_atom(wtab, a0)
    # paper: a0 = 3.1837 A, E_coh = -11.17 eV (EAM fit column)
    tol = GOLD["tolerances"]
    assert abs(a0 - GOLD["lattice_constant_A"]) < tol["lattice_constant_A"]
    assert abs(e0 - GOLD["cohesive_energy_eV"]) < tol["cohesive_energy_eV"]


def test_w_eam_elastic_constants(wtab):
    a0 = lattice_min(wtab)
    e0, v0 = energy_per_atom(wtab, a0)
    h = 2e-3

    def d2(eps):
        ep, _ = energy_per_atom(wtab, a0, h * eps)
        em, _ = energy_per_atom(wtab, a0, -h * eps)
        return (ep + em - 2 * e0) / (h * h) / v0 * EV_A3_TO_GPA

    c11 = d2(np.diag([1.0, 0, 0]))
    c11_c12 = d2(np.diag([1.0, 1.0, 0])) / 2.0
    c12 = c11_c12 - c11
    g = np.zeros((3, 3)); g[0, 1] = g[1, 0] = 0.5
    c44 = d2(g)
    B = (c11 + 2 * c12) / 3
    # paper: C11 508, C12 162, C44 140, B 277 GPa
    t = GOLD["tolerances"]["elastic_GPa"]
    assert abs(c11 - GOLD["C11_GPa"]) < t
    assert abs(c12 - GOLD["C12_GPa"]) < t
    assert abs(c44 - GOLD["C44_GPa"]) < t
    assert abs(B - GOLD["bulk_modulus_GPa"]) < t


def test_w_pair_continuity_at_bridge():
    # Phi^Fit and its first two derivatives are continuous at r_lo and r_hi
    for r0 in (w.W_EAM["r_lo"], w.W_EAM["r_hi"]):
        hh = 1e-7
        vm, dm = w.w_pair(np.array([r0 - hh]))
        vp, dp = w.w_pair(np.array([r0 + hh]))
        assert abs(vm[0] - vp[0]) < 1e-5 * max(1, abs(vp[0]))
        assert abs(dm[0] - dp[0]) < 1e-4 * max(1, abs(dp[0]))
        h2 = 1e-4
        def second(r):
            return (w.w_pair(np.array([r + h2]))[0][0] - 2 * w.w_pair(np.array([r]))[0][0]
                    + w.w_pair(np.array([r - h2]))[0][0]) / h2 ** 2
        s_in = second(r0 - 3 * h2) if r0 == w.W_EAM["r_hi"] else second(r0 + 3 * h2)
        s_out = second(r0 + 3 * h2) if r0 == w.W_EAM["r_hi"] else second(r0 - 3 * h2)
        assert abs(s_in - s_out) < 2e-2 * max(1.0, abs(s_in))


def test_density_maximum_at_rcut_and_zbl_length():
    p = w.W_EAM
    _, dz = w._knot_sum(np.array([p["r_cut_rho"]]), p["a_rho"], p["d_rho"])
    assert abs(dz[0]) < 1e-9
    a = 0.8854 * 0.529 / (74 ** 0.23 + 74 ** 0.23)
    assert abs(a - p["a_zbl"]) < 1e-6


def test_table_reproduces_cubic_exactly():
    # a clamped spline through a cubic with exact end slopes is that cubic
    f = lambda x: 0.3 - 1.2 * x + 0.7 * x ** 2 - 0.05 * x ** 3
    df = lambda x: -1.2 + 1.4 * x - 0.15 * x ** 2
    t = w.spline_table(f, 1.0, 5.5, 50, ("slope", df(1.0)), ("slope", df(5.5)))
    x = np.linspace(0.9, 5.5, 777)
    v, dv = evaluate(t.arrays(), x)
    assert np.allclose(v, f(x), atol=1e-12)
    assert np.allclose(dv, df(x), atol=1e-11)


def test_table_is_c2_at_knots():
    t = w.make_eam_tables("W", noise=0.01, seed=4).phi.arrays()
    c = t["coef"]
    dx = t["dx"]
    v_end = c[:-1, 0] + dx * (c[:-1, 1] + dx * (c[:-1, 2] + dx * c[:-1, 3]))
    d_end = c[:-1, 1] + dx * (2 * c[:-1, 2] + 3 * dx * c[:-1, 3])
    s_end = 2 * c[:-1, 2] + 6 * dx * c[:-1, 3]
    assert np.allclose(v_end, c[1:, 0], rtol=1e-10, atol=1e-10)
    assert np.allclose(d_end, c[1:, 1], rtol=1e-8, atol=1e-8)
    assert np.allclose(s_end, 2 * c[1:, 2], rtol=1e-6, atol=1e-6)


def test_eam_bond_gradient_matches_fd(wtab):
    rng = np.random.default_rng(1)
    d = rng.normal(0, 1, (40, 3))
    d *= (rng.uniform(2.2, 5.4, 40) / np.linalg.norm(d, axis=1))[:, None]
    E, _, g = wtab.energy_and_grad([d])
    h = 1e-6
    for j in range(0, 40, 7):
        for k in range(3):
            dp = d.copy(); dp[j, k] += h
            dm = d.copy(); dm[j, k] -= h
            fd = (wtab.energy_and_grad([dp])[0][0] - wtab.energy_and_grad([dm])[0][0]) / (2 * h)
            assert abs(fd - g[0][j, k]) < 1e-6 * max(1.0, abs(fd))


def test_table_beyond_end_branches():
    """Past the last knot a 'linear' table continues with its end value and
    slope (the embedding F), a 'zero' table is 0 (Phi and zeta, whose last
    knot is the cutoff); below the first knot the first cubic continues.
    Checked against the closed form of the tabulated cubic."""
    f = lambda x: 0.3 - 1.2 * x + 0.7 * x ** 2 - 0.05 * x ** 3
    df = lambda x: -1.2 + 1.4 * x - 0.15 * x ** 2
    x0, x1 = 1.0, 5.5
    t = w.spline_table(f, x0, x1, 50, ("slope", df(x0)), ("slope", df(x1))).arrays()
    x = np.array([5.5 + 1e-9, 5.6, 7.0, 12.25])
    v, dv = evaluate(t, x, "linear")
    assert np.allclose(v, f(x1) + df(x1) * (x - x1), rtol=0, atol=1e-11)
    assert np.allclose(dv, df(x1), rtol=0, atol=1e-11)
    v, dv = evaluate(t, x, "zero")
    assert np.all(v == 0.0) and np.all(dv == 0.0)
    xb = np.array([0.2, 0.5, 0.999])
    v, dv = evaluate(t, xb, "linear")
    assert np.allclose(v, f(xb), atol=1e-11) and np.allclose(dv, df(xb), atol=1e-10)
    # the EAM oracle takes the linear branch for F: an atom whose density is
    # past the end of the F table gets F_end + F'_end (rho - rho_end)
    orc = EamOracle(w.make_eam_tables("W", noise=0.01, seed=5))
    Ft = orc.F
    rho_end = Ft["x0"] + (Ft["n_knots"] - 1) * Ft["dx"]
    c = np.asarray(Ft["coef"])[-1]
    dx = Ft["dx"]
    F_end = c[0] + dx * (c[1] + dx * (c[2] + dx * c[3]))
    dF_end = c[1] + dx * (2 * c[2] + 3 * dx * c[3])
    d = np.array([[2.0, 0.0, 0.0]] * 40)      # forty bonds at 2 A: far above 2 rho_bulk
    rho = orc.density(d)
    assert rho > rho_end
    E, _, g = orc.energy_and_grad([d])
    ph, dph = evaluate(orc.phi, np.array([2.0]), "zero")
    z, dz = evaluate(orc.rho, np.array([2.0]), "zero")
    assert abs(E[0] - (F_end + dF_end * (rho - rho_end) + 0.5 * 40 * ph[0])) <= 1e-12 * abs(E[0])
    assert np.allclose(g[0][:, 0], dF_end * dz[0] + 0.5 * dph[0], rtol=1e-13, atol=0)
