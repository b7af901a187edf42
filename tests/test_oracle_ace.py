"""Pins of the ACE oracle: closed forms, brute force, invariances, FD."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle.ace import AceOracle
from paper_2505_12958_amd import workloads as w


@pytest.fixture(scope="module")
def ace3():
    return AceOracle(w.make_ace_model(6, 3, 3, 11, 58))


@pytest.fixture(scope="module")
def ace4():
    return AceOracle(w.make_ace_model(4, 3, 4, 12, 58))


def cluster(n, seed, rmin=2.2, rmax=5.3):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    return d * (rng.uniform(rmin, rmax, n) / np.linalg.norm(d, axis=1))[:, None]


def test_basis_counts():
    # counts of the canonical basis at the two model sizes
    f = w.enumerate_basis(6, 3, 3)
    assert [int(np.sum(f[:, 0] == k)) for k in (1, 2, 3, 4)] == [6, 84, 958, 0]
    f = w.enumerate_basis(8, 4, 4)
    assert [int(np.sum(f[:, 0] == k)) for k in (1, 2, 3, 4)] == [8, 180, 3976, 86806]


def test_chebyshev_and_cutoff(ace3):
    t = np.linspace(0.01, math.pi - 0.01, 50)
    r = (np.cos(t) + 1) * ace3.r_c / 2
    W = ace3.W.copy()
    ace3.W = np.zeros_like(W)
    try:
        for k in range(ace3.K):
            ace3.W[0, 0, :] = 0; ace3.W[0, 0, k] = 1
            R, _ = ace3.radial(r)
            fc = 0.5 * (1 + np.cos(math.pi * r / ace3.r_c))
            assert np.allclose(R[:, 0, 0], np.cos(k * t) * fc, atol=1e-13)
    finally:
        ace3.W = W
    R, dR = ace3.radial(np.array([ace3.r_c]))
    assert np.abs(R).max() < 1e-15 and np.abs(dR).max() < 1e-15


def test_radial_derivative_fd(ace3):
    r = np.linspace(1.5, 5.4, 30)
    _, dR = ace3.radial(r)
    h = 1e-6
    fd = (ace3.radial(r + h)[0] - ace3.radial(r - h)[0]) / (2 * h)
    assert np.allclose(dR, fd, atol=1e-9)


def test_nu2_invariant_closed_form(ace3):
    # sum_m A_{n1 l m} A_{n2 l m} = (2l+1)/(4pi) sum_{j,k} R_{n1 l}(r_j) R_{n2 l}(r_k) P_l(cos t_jk)
    d = cluster(25, 1)
    A, _ = ace3.atomic_basis(d[None], np.ones((1, 25), bool))
    A = A[0]
    r = np.linalg.norm(d, axis=1)
    R, _ = ace3.radial(r)
    u = d / r[:, None]
    c = np.clip(u @ u.T, -1, 1)
    for l in range(ace3.l_max + 1):
        Pl = np.polynomial.legendre.legval(c, [0] * l + [1])
        for n1, n2 in [(0, 0), (1, 3), (5, 2)]:
            lhs = np.sum(A[n1, l * l:(l + 1) ** 2] * A[n2, l * l:(l + 1) ** 2])
            rhs = (2 * l + 1) / (4 * math.pi) * R[:, n1, l] @ Pl @ R[:, n2, l]
            assert abs(lhs - rhs) < 1e-13 * max(1, abs(rhs))


def test_nu2_basis_value_is_coupled_invariant(ace3):
    # B for nu=2 equals (-1)^l/sqrt(2l+1) sum_m A_{n1lm} A_{n2lm}
    d = cluster(30, 2)
    B = ace3.basis_values([d])[0]
    A, _ = ace3.atomic_basis(d[None], np.ones((1, 30), bool))
    A = A[0]
    for v, f in enumerate(ace3.funcs):
        if f[0] == 2:
            n1, l, n2 = f[1], f[2], f[3]
            ref = (-1) ** l / math.sqrt(2 * l + 1) * np.sum(A[n1, l * l:(l + 1) ** 2] * A[n2, l * l:(l + 1) ** 2])
            assert abs(B[v] - ref) < 1e-14


@pytest.mark.parametrize("which", ["ace3", "ace4"])
def test_rotation_translation_permutation_invariance(which, request):
    orc = request.getfixturevalue(which)
    d = cluster(40, 3)
    rot = Rotation.random(random_state=7).as_matrix()
    perm = np.random.default_rng(8).permutation(40)
    B0 = orc.basis_values([d])[0]
    B1 = orc.basis_values([d @ rot.T])[0]
    B2 = orc.basis_values([d[perm]])[0]
    scale = np.abs(B0).max()
    assert np.abs(B1 - B0).max() < 1e-12 * scale
    assert np.abs(B2 - B0).max() < 1e-13 * scale
    E0, g0, _, _ = orc.energy_and_grad([d])
    E1, g1, _, _ = orc.energy_and_grad([d @ rot.T])
    assert abs(E1[0] - E0[0]) < 1e-13
    # gradients rotate with the frame (covariance)
    assert np.allclose(g1[0], g0[0] @ rot.T, atol=1e-13)


@pytest.mark.parametrize("which", ["ace3", "ace4"])
def test_bond_gradient_fd(which, request):
    orc = request.getfixturevalue(which)
    d = cluster(30, 4)
    E, g, phi, _ = orc.energy_and_grad([d])
    assert abs(phi[0, 1]) > 1e-4                      # away from the guard's kink
    h = 1e-5
    for j in range(0, 30, 6):
        for k in range(3):
            dp = d.copy(); dp[j, k] += h
            dm = d.copy(); dm[j, k] -= h
            fd = (orc.energy_and_grad([dp])[0][0] - orc.energy_and_grad([dm])[0][0]) / (2 * h)
            assert abs(fd - g[0][j, k]) < 1e-9 * max(1e-3, abs(g[0]).max()), (j, k)


def test_embedding_sign_branch():
    # a model whose phi2 is negative uses sqrt(|phi2| + 1e-6) with sgn = -1
    m = w.make_ace_model(3, 2, 2, 13, 58)
    orc = AceOracle(m)
    d = cluster(20, 5)
    _, _, phi, _ = orc.energy_and_grad([d])
    if phi[0, 1] > 0:
        m.c2 = -m.c2
        orc = AceOracle(m)
    E, g, phi, _ = orc.energy_and_grad([d])
    assert phi[0, 1] < 0
    assert abs(E[0] - (phi[0, 0] + math.sqrt(abs(phi[0, 1]) + 1e-6))) < 1e-15
    h = 1e-6
    dp = d.copy(); dp[3, 1] += h
    dm = d.copy(); dm[3, 1] -= h
    fd = (orc.energy_and_grad([dp])[0][0] - orc.energy_and_grad([dm])[0][0]) / (2 * h)
    assert abs(fd - g[0][3, 1]) < 1e-8
