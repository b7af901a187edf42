"""Pin of the oracle's product basis (nu = 1..4) by an independent evaluation
in the complex spherical basis.

The ACE basis of the section "Atomic cluster expansion" is a set of rotation
invariants built from the atomic basis A_nlm.  Written in complex harmonics
Y_l^mu (Condon-Shortley phase, scipy's sph_harm_y) and the complex
Clebsch-Gordan coefficients (sympy, exact), the real-basis definitions used by
the oracle are equivalent to

  A^c_{n l mu}      = sum_j R_nl(r_j) Y_l^mu(u_j)
  AA^c_{(a,b),L,mu} = sum_{mu1} <l_a mu1 l_b (mu - mu1) | L mu> A^c_{a,mu1} A^c_{b,mu-mu1}
  nu=1  B = A^c_{n 0 0}
  nu=2  B = AA^c_{(a,b),0,0}
  nu=3  B = sum_mu AA^c_{(a,b),L,mu} conj(A^c_{d,mu})
  nu=4  B = sum_mu AA^c_{(a,b),L,mu} conj(AA^c_{(c,d),L,mu})

(the real transform U is unitary with U^T U = (-1)^mu delta_{mu,-mu'}, and
A^c_{-mu} = (-1)^mu conj(A^c_mu) for real radial functions, so the real
contraction sum_M X_M Y_M equals the Hermitian product above).  Nothing here
calls the oracle's harmonics, coupling coefficients, radial basis or
channel bookkeeping: the radial basis is retyped from the closed form
T_k(x) = cos(k arccos x), each function tuple is read as the model file
states it, and a mis-paired channel, a wrong coupled rank or a transposed
operand in the oracle changes B.
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y
from sympy.physics.wigner import clebsch_gordan

from oracle.ace import AceOracle
from paper_2505_12958_amd import workloads as w


def cluster(n, seed, rmin=2.2, rmax=5.3):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    return d * (rng.uniform(rmin, rmax, n) / np.linalg.norm(d, axis=1))[:, None]


_CG = {}


def cg(l1, m1, l2, m2, L, M):
    key = (l1, m1, l2, m2, L, M)
    if key not in _CG:
        _CG[key] = float(clebsch_gordan(l1, l2, L, m1, m2, M))
    return _CG[key]


def complex_basis_values(model, d):
    """All B_v of the model's function list for one atom with bonds d[j, 3]."""
    n_max, l_max, K, rc = model.n_max, model.l_max, model.K, model.r_c
    W = np.asarray(model.W).reshape(n_max, l_max + 1, K)
    r = np.linalg.norm(d, axis=1)
    x = 2.0 * r / rc - 1.0
    g = np.stack([np.cos(k * np.arccos(x)) for k in range(K)], 1) * (0.5 * (1 + np.cos(np.pi * r / rc)))[:, None]
    R = np.einsum("jk,nlk->jnl", g, W)
    theta = np.arccos(np.clip(d[:, 2] / r, -1, 1))
    phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
    Ac = {}
    for n in range(n_max):
        for l in range(l_max + 1):
            for mu in range(-l, l + 1):
                Ac[n, l, mu] = np.sum(R[:, n, l] * sph_harm_y(l, mu, theta, phi))

    def AA(na, la, nb, lb, L):
        out = np.zeros(2 * L + 1, dtype=complex)
        for mu in range(-L, L + 1):
            s = 0j
            for mu1 in range(-la, la + 1):
                mu2 = mu - mu1
                if abs(mu2) <= lb:
                    s += cg(la, mu1, lb, mu2, L, mu) * Ac[na, la, mu1] * Ac[nb, lb, mu2]
            out[mu + L] = s
        return out

    out = np.zeros(len(model.funcs), dtype=complex)
    for v, f in enumerate(np.asarray(model.funcs)):
        nu, L = int(f[0]), int(f[9])
        if nu == 1:
            out[v] = Ac[f[1], 0, 0]
        elif nu == 2:
            out[v] = AA(f[1], f[2], f[3], f[4], 0)[0]
        elif nu == 3:
            a = AA(f[1], f[2], f[3], f[4], L)
            dvec = np.array([Ac[f[5], f[6], mu] for mu in range(-L, L + 1)])
            out[v] = np.sum(a * np.conj(dvec))
        else:
            out[v] = np.sum(AA(f[1], f[2], f[3], f[4], L) * np.conj(AA(f[5], f[6], f[7], f[8], L)))
    return out


@pytest.fixture(scope="module")
def small4():
    # nu <= 4 with every coupled rank up to 2 l_max, and distinct n on each index
    return w.make_ace_model(3, 2, 4, 21, 58)


def test_model_covers_every_order(small4):
    f = np.asarray(small4.funcs)
    counts = [int(np.sum(f[:, 0] == k)) for k in (1, 2, 3, 4)]
    assert min(counts) > 0, counts
    assert set(np.unique(f[f[:, 0] == 4, 9])) == {0, 1, 2, 3, 4}


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_product_basis_equals_complex_definition(small4, seed):
    d = cluster(9 + seed, 40 + seed)
    ref = complex_basis_values(small4, d)
    # every invariant is real
    assert np.abs(ref.imag).max() <= 1e-13 * max(1.0, np.abs(ref.real).max())
    B = AceOracle(small4).basis_values([d])[0]
    f = np.asarray(small4.funcs)
    for nu in (1, 2, 3, 4):
        sel = f[:, 0] == nu
        scale = max(1e-300, np.abs(ref.real[sel]).max())
        err = np.abs(B[sel] - ref.real[sel]).max() / scale
        assert err <= 1e-12, (nu, err)


def test_pin_detects_a_mispaired_nu4_channel(small4):
    """A planted mistake in the oracle (nu = 4 contracting the first coupled
    pair with itself instead of with the second) fails the pin."""
    d = cluster(10, 44)
    ref = complex_basis_values(small4, d).real
    orc = AceOracle(small4)
    f = np.asarray(small4.funcs)
    # the product terms of nu=4 functions: point the second factor at the first
    term_fn = orc.S_b.tocoo()
    nu4_terms = term_fn.row[f[term_fn.col, 0] == 4]
    bq = orc.b_q.copy()
    bq[nu4_terms] = orc.b_p[nu4_terms]
    orc.b_q = bq
    B = orc.basis_values([d])[0]
    sel = f[:, 0] == 4
    assert np.abs(B[sel] - ref[sel]).max() > 1e-6 * np.abs(ref[sel]).max()
