"""Clebsch-Gordan coefficients in the real-harmonic basis (oracle, FP64).

Complex <l1 m1 l2 m2 | L M> from Racah's closed-form sum, evaluated exactly
with rational arithmetic.  Real harmonics relate to complex ones by
Y_real_m = sum_mu U_{m mu} Y^mu with U from the real convention of ``ylm``:
U_{00} = 1; m > 0: U_{m,m} = (-1)^m/sqrt2, U_{m,-m} = 1/sqrt2;
m < 0, k = |m|: U_{m,k} = -i(-1)^k/sqrt2, U_{m,-k} = i/sqrt2.
The coupling coefficient of two real tensors into a real rank-L tensor is

    C^{l1 l2 L}_{m1 m2 M} = sum U^L_{M mu} conj(U^{l1}_{m1 mu1}) conj(U^{l2}_{m2 mu2})
                             <l1 mu1 l2 mu2 | L mu>,

real whenever l1 + l2 + L is even (the only couplings the model uses).
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np


def cg_complex(j1, m1, j2, m2, J, M):
    """<j1 m1 j2 m2 | J M> (integer spins), Racah's formula, exact."""
    if m1 + m2 != M or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    if J < abs(j1 - j2) or J > j1 + j2:
        return 0.0
    f = math.factorial
    pre = Fraction((2 * J + 1) * f(J + j1 - j2) * f(J - j1 + j2) * f(j1 + j2 - J), f(j1 + j2 + J + 1))
    pre *= f(J + M) * f(J - M) * f(j1 - m1) * f(j1 + m1) * f(j2 - m2) * f(j2 + m2)
    s = Fraction(0)
    for k in range(0, j1 + j2 - J + 1):
        args = [k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k]
        if min(args) < 0:
            continue
        den = 1
        for a in args:
            den *= f(a)
        s += Fraction((-1) ** k, den)
    val = math.sqrt(pre) * float(s) if pre.denominator == 1 else math.sqrt(float(pre)) * float(s)
    return val


def u_matrix(l):
    """U[m + l, mu + l] mapping complex to real harmonics."""
    U = np.zeros((2 * l + 1, 2 * l + 1), dtype=np.complex128)
    s = 1.0 / math.sqrt(2.0)
    for m in range(-l, l + 1):
        if m == 0:
            U[l, l] = 1.0
        elif m > 0:
            U[m + l, m + l] = (-1) ** m * s
            U[m + l, -m + l] = s
        else:
            k = -m
            U[m + l, k + l] = -1j * (-1) ** k * s
            U[m + l, -k + l] = 1j * s
    return U


@lru_cache(maxsize=None)
def cg_real(l1, l2, L):
    """Real coupling tensor C[m1+l1, m2+l2, M+L] (complex dtype for inspection)."""
    Cc = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * L + 1))
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            M = m1 + m2
            if abs(M) <= L:
                Cc[m1 + l1, m2 + l2, M + L] = cg_complex(l1, m1, l2, m2, L, M)
    U1, U2, UL = u_matrix(l1), u_matrix(l2), u_matrix(L)
    return np.einsum("Mc,ia,jb,abc->ijM", UL, U1.conj(), U2.conj(), Cc)


def cg_real_checked(l1, l2, L):
    """Real part of cg_real, asserting the imaginary part vanishes."""
    C = cg_real(l1, l2, L)
    if np.max(np.abs(C.imag)) > 1e-12:
        raise ValueError(f"coupling ({l1},{l2},{L}) is not real")
    return C.real
