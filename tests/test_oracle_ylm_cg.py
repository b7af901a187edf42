"""Pins of the oracle's real harmonics and coupling coefficients against
textbook identities and independent libraries (scipy, sympy)."""
import math

import numpy as np
import pytest

from oracle import cg, ylm


def sphere_quadrature(deg):
    # Gauss-Legendre in z times a uniform grid in phi: exact for degree <= deg
    z, wz = np.polynomial.legendre.leggauss(deg // 2 + 2)
    nphi = deg + 2
    phi = 2 * math.pi * np.arange(nphi) / nphi
    Z, P = np.meshgrid(z, phi, indexing="ij")
    s = np.sqrt(1 - Z ** 2)
    u = np.stack([s * np.cos(P), s * np.sin(P), Z], -1).reshape(-1, 3)
    wts = (wz[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    return u, wts


def test_orthonormal():
    L = 6
    u, wts = sphere_quadrature(2 * L)
    Y = ylm.real_ylm(u, L)
    G = (Y * wts[:, None]).T @ Y
    assert np.abs(G - np.eye((L + 1) ** 2)).max() < 1e-13


def test_low_orders_closed_form():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(20, 3))
    Y = ylm.real_ylm(d, 2)
    u = d / np.linalg.norm(d, axis=1)[:, None]
    assert np.allclose(Y[:, 0], 0.5 / math.sqrt(math.pi))
    c = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 1:4], c * u[:, [1, 2, 0]])
    # Y_{2,0} = sqrt(5/16pi)(3z^2-1), Y_{2,2} = sqrt(15/16pi)(x^2-y^2), Y_{2,-2} = sqrt(15/4pi) x y
    assert np.allclose(Y[:, 6], math.sqrt(5 / (16 * math.pi)) * (3 * u[:, 2] ** 2 - 1))
    assert np.allclose(Y[:, 8], math.sqrt(15 / (16 * math.pi)) * (u[:, 0] ** 2 - u[:, 1] ** 2))
    assert np.allclose(Y[:, 4], math.sqrt(15 / (4 * math.pi)) * u[:, 0] * u[:, 1])


def test_addition_theorem():
    rng = np.random.default_rng(1)
    a, b = rng.normal(size=(2, 30, 3))
    Ya, Yb = ylm.real_ylm(a, 6), ylm.real_ylm(b, 6)
    ua = a / np.linalg.norm(a, axis=1)[:, None]
    ub = b / np.linalg.norm(b, axis=1)[:, None]
    c = np.sum(ua * ub, 1)
    for l in range(7):
        s = np.sum(Ya[:, l * l:(l + 1) ** 2] * Yb[:, l * l:(l + 1) ** 2], 1)
        Pl = np.polynomial.legendre.legval(c, [0] * l + [1])
        assert np.allclose(s, (2 * l + 1) / (4 * math.pi) * Pl, atol=1e-13)


def test_against_scipy():
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(2)
    d = rng.normal(size=(25, 3))
    r = np.linalg.norm(d, axis=1)
    theta = np.arccos(d[:, 2] / r)
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = ylm.real_ylm(d, 5)
    for l in range(6):
        for m in range(-l, l + 1):
            if m == 0:
                ref = sph_harm_y(l, 0, theta, phi).real
            elif m > 0:
                ref = math.sqrt(2) * (-1) ** m * sph_harm_y(l, m, theta, phi).real
            else:
                ref = math.sqrt(2) * (-1) ** m * sph_harm_y(l, -m, theta, phi).imag
            assert np.allclose(Y[:, l * l + l + m], ref, atol=1e-12), (l, m)


def test_gradient_fd():
    rng = np.random.default_rng(3)
    d = rng.normal(size=(10, 3)) * 2
    _, G = ylm.real_ylm(d, 5, grad=True)
    h = 1e-6
    for k in range(3):
        dp = d.copy(); dp[:, k] += h
        dm = d.copy(); dm[:, k] -= h
        fd = (ylm.real_ylm(dp, 5) - ylm.real_ylm(dm, 5)) / (2 * h)
        assert np.allclose(G[..., k], fd, atol=1e-8)


def test_complex_cg_against_sympy():
    from sympy.physics.quantum.cg import CG
    rng = np.random.default_rng(4)
    for _ in range(60):
        j1, j2 = rng.integers(0, 5, 2)
        J = rng.integers(abs(j1 - j2), j1 + j2 + 1)
        m1 = rng.integers(-j1, j1 + 1)
        m2 = rng.integers(-j2, j2 + 1)
        M = m1 + m2
        if abs(M) > J:
            continue
        ref = float(CG(int(j1), int(m1), int(j2), int(m2), int(J), int(M)).doit())
        assert abs(cg.cg_complex(int(j1), int(m1), int(j2), int(m2), int(J), int(M)) - ref) < 1e-14


@pytest.mark.parametrize("l1,l2,L", [(0, 0, 0), (1, 1, 0), (1, 1, 2), (1, 2, 1), (1, 2, 3),
                                     (2, 2, 2), (2, 3, 3), (3, 3, 4), (4, 4, 4), (4, 4, 8), (3, 4, 5)])
def test_real_cg_real_orthonormal_and_product_identity(l1, l2, L):
    C = cg.cg_real(l1, l2, L)
    assert np.abs(C.imag).max() < 1e-14
    C = C.real
    M = C.reshape(-1, 2 * L + 1)
    assert np.abs(M.T @ M - np.eye(2 * L + 1)).max() < 1e-13
    # sum C Y_l1 Y_l2 = kappa Y_L with kappa = sqrt((2l1+1)(2l2+1)/(4pi(2L+1))) <l1 0 l2 0|L 0>
    from sympy.physics.quantum.cg import CG
    k = math.sqrt((2 * l1 + 1) * (2 * l2 + 1) / (4 * math.pi * (2 * L + 1))) * float(
        CG(l1, 0, l2, 0, L, 0).doit())
    rng = np.random.default_rng(5)
    u = rng.normal(size=(12, 3))
    Y = ylm.real_ylm(u, max(l1, l2, L))
    lhs = np.einsum("abM,na,nb->nM", C, Y[:, l1 * l1:(l1 + 1) ** 2], Y[:, l2 * l2:(l2 + 1) ** 2])
    assert np.allclose(lhs, k * Y[:, L * L:(L + 1) ** 2], atol=1e-13)


def test_odd_coupling_is_imaginary():
    C = cg.cg_real(1, 1, 1)
    assert np.abs(C.real).max() < 1e-14 and np.abs(C.imag).max() > 0.1
