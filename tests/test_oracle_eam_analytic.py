"""Pins of the closed-form W EAM oracle against what the paper prints
(appendix "AP potential for tungsten": the 'fit' column of the table of
tungsten potential properties; the bridge's continuity of Phi and its first
two derivatives; the density's maximum at r_cut) and against the
generator's independently coded tables of the same form."""
import json
import math
import os

import numpy as np
import pytest

from oracle.eam import EamOracle
from oracle.eam_analytic import AnalyticWEam
from oracle.geometry import Systems
from paper_2505_12958_amd import workloads as w
from paper_2505_12958_amd.workloads import lattice_points

EV_A3_TO_GPA = 160.21766208
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "w_eam_fit_properties.json")))


@pytest.fixture(scope="module")
def weam():
    return AnalyticWEam(dict(w.W_EAM, zbl=w.ZBL_C))


def energy_per_atom(orc, a, eps=None, n=4):
    p = lattice_points("bcc", (n, n, n), a)
    H = np.eye(3) * n * a
    if eps is not None:
        F = np.eye(3) + eps
        p = p @ F.T
        H = H @ F.T
    S = Systems(p, H[None], [0, len(p)], (True, True, True), 5.5)
    E, _, _ = orc.energy_and_grad([x[1] for x in S.neighbour_lists()])
    return E.sum() / len(p), abs(np.linalg.det(H)) / len(p)


def test_fit_properties_of_the_paper(weam):
    lo, hi = 3.15, 3.22
    g = (math.sqrt(5) - 1) / 2
    for _ in range(60):
        x1, x2 = hi - g * (hi - lo), lo + g * (hi - lo)
        if energy_per_atom(weam, x1)[0] < energy_per_atom(weam, x2)[0]:
            hi = x2
        else:
            lo = x1
    a0 = 0.5 * (lo + hi)
    e0, v0 = energy_per_atom(weam, a0)
    tol = GOLD["tolerances"]
    assert abs(a0 - GOLD["lattice_constant_A"]) < tol["lattice_constant_A"]
    assert abs(e0 - GOLD["cohesive_energy_eV"]) < tol["cohesive_energy_eV"]
    h = 2e-3

    def d2(eps):
        ep, _ = energy_per_atom(weam, a0, h * eps)
        em, _ = energy_per_atom(weam, a0, -h * eps)
        return (ep + em - 2 * e0) / (h * h) / v0 * EV_A3_TO_GPA

    c11 = d2(np.diag([1.0, 0, 0]))
    c12 = d2(np.diag([1.0, 1.0, 0])) / 2.0 - c11
    s = np.zeros((3, 3)); s[0, 1] = s[1, 0] = 0.5
    c44 = d2(s)
    t = tol["elastic_GPa"]
    for val, key in ((c11, "C11_GPa"), (c12, "C12_GPa"), (c44, "C44_GPa"),
                     ((c11 + 2 * c12) / 3, "bulk_modulus_GPa")):
        assert abs(val - GOLD[key]) < t, (key, val)


def test_bridge_continuity_and_density_maximum(weam):
    p = w.W_EAM
    for r0 in (p["r_lo"], p["r_hi"]):
        hh = 1e-8
        vm, dm = weam.pair(np.array([r0 - hh]))
        vp, dp = weam.pair(np.array([r0 + hh]))
        assert abs(vm[0] - vp[0]) < 1e-5 * abs(vp[0])
        assert abs(dm[0] - dp[0]) < 1e-5 * abs(dp[0])

        def second(r):
            return (weam.pair(np.array([r + 1e-5]))[1][0] - weam.pair(np.array([r - 1e-5]))[1][0]) / 2e-5
        assert abs(second(r0 - 1e-4) - second(r0 + 1e-4)) < 2e-3 * abs(second(r0 + 1e-4))
    # zeta_0 has its maximum at r_cut: zero slope there, held constant below
    _, dz = weam._knots(np.array([p["r_cut_rho"]]), p["a_rho"], p["d_rho"])
    assert abs(dz[0]) < 1e-9
    z, dzr = weam.density(np.array([1.5, 2.0, p["r_cut_rho"]]))
    assert np.all(z == z[-1]) and np.all(dzr == 0.0)
    # the knot sums vanish beyond their last knots, inside the cutoff
    v, dv = weam.pair(np.array([max(p["d_phi"]) + 1e-9, 5.5]))
    assert np.all(v == 0.0) and np.all(dv == 0.0)
    # the embedding's square-root branch and its guard
    x = np.array([0.0, 1e-12, 3.0])
    v, dv = weam.embed(x)
    a1, a2 = p["a_xi"]
    assert np.allclose(v, a1 * np.sqrt(x) + a2 * x * x + p["d_xi"], rtol=1e-14, atol=1e-14)
    assert dv[0] == 0.0 and np.isclose(dv[2], 0.5 * a1 / math.sqrt(3.0) + 2 * a2 * 3.0, rtol=1e-14)


def test_agrees_with_the_generators_tables(weam):
    tab = EamOracle(w.make_eam_tables("W", noise=0.0))
    # environments of a strained, jittered BCC cell: densities inside the
    # tables' domain [0, 2 rho_bulk]
    p = lattice_points("bcc", (4, 4, 4), 3.165) * 0.97
    p = p + np.random.default_rng(3).normal(0, 0.1, p.shape)
    L = 4 * 3.165 * 0.97
    S = Systems(np.mod(p, L), np.diag([L, L, L])[None], [0, len(p)], (True, True, True), 5.5)
    d_list = [r[1] for r in S.neighbour_lists()]
    Ea, ra, ga = weam.energy_and_grad(d_list)
    Et, rt, gt = tab.energy_and_grad(d_list)
    assert np.abs(Ea - Et).max() < 1e-4 * np.abs(Ea).max()
    assert np.abs(ra - rt).max() < 1e-4 * np.abs(ra).max()
    # bond gradients away from the density's kink at r_cut, where zeta'' jumps
    # and the cubic table smooths it over a knot interval
    dx = tab.rho["dx"]
    far = [i for i, d in enumerate(d_list)
           if np.min(np.abs(np.linalg.norm(d, axis=1) - w.W_EAM["r_cut_rho"])) > 2 * dx]
    assert len(far) > len(d_list) // 2
    # (the cubic tables interpolate derivatives to ~1e-3 near the knots of the
    # pair sum, where the third derivative jumps)
    assert max(np.abs(ga[i] - gt[i]).max() for i in far) < 3e-3 * max(np.abs(a).max() for a in ga)
