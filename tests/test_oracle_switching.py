"""Pins of the dynamic-switching oracle (appendix "Switching function": the
CSP of the 14 nearest neighbours and the table of the adaptive-precision
model's parameters): closed forms of each step and of their composition."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle.geometry import Systems
from oracle.switching import (DynamicSwitching, SwitchParams, csp_all, csp_of, detection, ramp,
                              snap, spread, transition)
from paper_2505_12958_amd.workloads import lattice_points


def cell(kind, n, a, jitter=0.0, seed=0):
    p = lattice_points(kind, (n, n, n), a)
    if jitter:
        p = p + np.random.default_rng(seed).normal(0, jitter, p.shape)
    L = n * a
    p = np.mod(p, L)
    return Systems(p, np.diag([L, L, L])[None], [0, len(p)], (True, True, True), 5.5)


def test_csp_zero_on_perfect_bcc_and_fcc():
    S = cell("bcc", 4, 3.165)
    rows = S.neighbour_lists()
    assert all(len(r[0]) == 58 for r in rows)          # 8 + 6 + 12 + 24 + 8
    assert np.abs(csp_all(S, rows, 14)).max() < 1e-24
    F = cell("fcc", 4, 3.615)
    assert np.abs(csp_all(F, F.neighbour_lists(), 12)).max() < 1e-24


def test_csp_of_one_displaced_neighbour_is_its_squared_displacement():
    S = cell("bcc", 4, 3.165)
    js, d = S.neighbours_of(0)
    r2 = np.sum(d * d, 1)
    near = np.argsort(r2, kind="stable")[:14]
    delta = np.array([0.031, -0.017, 0.022])
    for k in near[[0, 9]]:                              # a first- and a second-shell neighbour
        dd = d.copy()
        dd[k] = dd[k] + delta
        assert abs(csp_of(dd, 14) - np.dot(delta, delta)) <= 1e-12 * np.dot(delta, delta)


def test_csp_invariances():
    S = cell("bcc", 4, 3.165, jitter=0.08, seed=3)
    js, d = S.neighbours_of(5)
    c = csp_of(d)
    assert c > 0.01
    R = Rotation.random(random_state=4).as_matrix()
    assert abs(csp_of(d @ R.T) - c) <= 1e-12 * c
    perm = np.random.default_rng(1).permutation(len(d))
    assert abs(csp_of(d[perm]) - c) <= 1e-12 * c
    # only the 14 nearest count: adding far neighbours changes nothing
    far = np.vstack([d, d[:3] * 1.8])
    assert csp_of(far) == c
    # fewer than 14 neighbours: the largest value a full set could have
    assert csp_of(d[:13]) == 7 * 11.0 * 11.0


def test_ramp_and_transition_closed_forms():
    assert ramp(1.5, 1.5, 1.6) == 0.0 and ramp(1.6, 1.5, 1.6) == 1.0
    assert abs(ramp(1.55, 1.5, 1.6) - 0.5) < 1e-12
    assert ramp(0.2, 1.5, 1.6) == 0.0 and ramp(9.0, 1.5, 1.6) == 1.0
    c = np.linspace(1.5, 1.6, 101)
    assert np.all(np.diff(ramp(c, 1.5, 1.6)) >= 0)
    assert transition(4.0, 4.0, 12.0) == 1.0 and transition(12.0, 4.0, 12.0) == 0.0
    assert abs(transition(8.0, 4.0, 12.0) - 0.5) < 1e-12
    h = 1e-6                                            # zero slope at both ends (C^1)
    assert abs(transition(4.0 + h, 4.0, 12.0) - 1.0) < 1e-10
    assert abs(transition(12.0 - h, 4.0, 12.0)) < 1e-10
    assert abs(ramp(1.5 + 1e-7, 1.5, 1.6)) < 1e-10
    assert np.array_equal(snap([0.0, 0.009, 0.01, 0.5, 0.99, 0.991, 1.0], 0.01),
                          [0.0, 0.0, 0.01, 0.5, 0.99, 1.0, 1.0])


def test_spread_from_one_source_against_explicit_images():
    S = cell("bcc", 9, 3.165, jitter=0.05, seed=2)       # 28.5 A: > 2 r_hi
    p = SwitchParams()
    mu0 = np.zeros(S.n_atoms)
    src = 17
    mu0[src] = 0.7
    mu = spread(S, mu0, p)
    L = S.box[0][0][0]
    shifts = np.array([[x, y, z] for x in (-1, 0, 1) for y in (-1, 0, 1) for z in (-1, 0, 1)]) * L
    for i in range(0, S.n_atoms, 7):
        r = np.min(np.linalg.norm(S.pos[i][None, :] + shifts - S.pos[src][None, :], axis=1))
        g = 1.0 if r <= 4.0 else (0.5 * (1 + math.cos(math.pi * (r - 4.0) / 8.0)) if r < 12.0 else 0.0)
        assert abs(mu[i] - 0.7 * g) < 1e-12, (i, r)
    # a second, weaker source never lowers the first one's zone (max)
    mu0[src + 1] = 0.1
    assert np.all(spread(S, mu0, p) >= mu - 1e-15)


def test_fixed_zones_override_the_detection():
    S = cell("bcc", 6, 3.165)
    c = np.full(S.n_atoms, 5.0)                          # everything detected as precise
    centre = S.pos.mean(0)
    p = SwitchParams(centre=tuple(centre), r_precise=5.0, z_surface_min=float(np.quantile(S.pos[:, 2], 0.8)))
    mu0 = detection(S.pos, c, p)
    inside = np.linalg.norm(S.pos - centre, axis=1) <= 5.0
    surf = (S.pos[:, 2] >= p.z_surface_min) & ~inside
    assert np.all(mu0[inside] == 1.0) and np.all(mu0[surf] == 0.0) and np.all(mu0[~inside & ~surf] == 1.0)
    c[:] = 0.0                                           # nothing detected: only the ball stays
    assert np.array_equal(detection(S.pos, c, p), inside.astype(float))


def test_time_averages_follow_their_recursions():
    S0 = cell("bcc", 5, 3.165, jitter=0.06, seed=5)
    S1 = cell("bcc", 5, 3.165, jitter=0.06, seed=6)
    p = SwitchParams(csp_lo=0.05, csp_hi=0.15, n_csp_avg=7, n_lambda_avg=5, r_lo=2.0, r_hi=4.0)
    sw = DynamicSwitching(p)
    rows0, rows1 = S0.neighbour_lists(), S1.neighbour_lists()
    lam0 = sw.update(S0, rows0)
    c0, c1 = csp_all(S0, rows0), csp_all(S1, rows1)
    assert np.array_equal(sw.c_avg, c0)
    mu_first = spread(S0, detection(S0.pos, c0, p), p)
    assert np.array_equal(lam0, snap(mu_first, p.dlambda_min))
    for n in range(1, 6):
        lam = sw.update(S1, rows1)
        ref = c1 + (c0 - c1) * (1 - 1 / 7) ** n
        assert np.allclose(sw.c_avg, ref, rtol=0, atol=1e-13)
    assert np.all((lam >= 0) & (lam <= 1))
    # the lambda average after the last step, from its definition
    m_prev = sw.m_avg.copy()
    lam = sw.update(S1, rows1)
    c_next = sw.c_avg
    mu = spread(S1, detection(S1.pos, c_next, p), p)
    assert np.allclose(sw.m_avg, m_prev + (mu - m_prev) / 5, atol=1e-15)
    assert np.array_equal(lam, snap(sw.m_avg, p.dlambda_min))
