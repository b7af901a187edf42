"""Real orthonormal spherical harmonics and their gradients (oracle, FP64).

Convention: complex Y_l^m carry the Condon-Shortley phase.  The real
harmonics are Y_{l0} = Y_l^0, Y_{l,m>0} = sqrt2 (-1)^m Re Y_l^m and
Y_{l,m<0} = sqrt2 (-1)^m Im Y_l^{|m|}.  For a unit vector u = (x, y, z),
Y_l^m = (-1)^m N_lm P_l^{(m)}(z) (x + i y)^m with P_l^{(m)} the m-th
derivative of the Legendre polynomial and
N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), hence

    Y_{l,m>0} = sqrt2 N_lm P_l^{(m)}(z) Re (x+iy)^m,
    Y_{l,0}   =       N_l0 P_l(z),
    Y_{l,m<0} = sqrt2 N_l|m| P_l^{(|m|)}(z) Im (x+iy)^|m|.

Index: lm = l*l + l + m.  The gradient with respect to a (non-unit) bond
vector d is (I - u u^T) grad_u Y / |d|, grad_u taken of the polynomial above.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def _legendre_derivs(l_max):
    """Power-series coefficients of P_l^{(m)} for 0 <= m <= l+1 <= l_max+1."""
    out = {}
    for l in range(l_max + 1):
        c = npleg.leg2poly([0] * l + [1])
        for m in range(0, l + 2):
            out[(l, m)] = nppoly.polyder(c, m) if m > 0 else c
    return out


_CACHE = {}


def real_ylm(d, l_max, grad=False):
    """Y[..., lm] of bond vectors d[..., 3]; with grad=True also dY/dd[..., lm, 3]."""
    key = l_max
    if key not in _CACHE:
        _CACHE[key] = _legendre_derivs(l_max)
    P = _CACHE[key]
    d = np.asarray(d, dtype=np.float64)
    r = np.sqrt(np.sum(d * d, axis=-1))
    u = d / r[..., None]
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    w = x + 1j * y
    nlm = (l_max + 1) ** 2
    Y = np.zeros(d.shape[:-1] + (nlm,))
    G = np.zeros(d.shape[:-1] + (nlm, 3)) if grad else None
    wpow = [np.ones_like(w)]
    for m in range(1, l_max + 1):
        wpow.append(wpow[-1] * w)
    for l in range(l_max + 1):
        for m in range(0, l + 1):
            N = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            q = nppoly.polyval(z, P[(l, m)])
            dq = nppoly.polyval(z, P[(l, m + 1)]) if m + 1 <= l else np.zeros_like(z)
            if m == 0:
                Y[..., l * l + l] = N * q
                if grad:
                    G[..., l * l + l, 2] = N * dq
                continue
            s = math.sqrt(2.0) * N
            re, im = wpow[m].real, wpow[m].imag
            Y[..., l * l + l + m] = s * q * re
            Y[..., l * l + l - m] = s * q * im
            if grad:
                re1, im1 = wpow[m - 1].real, wpow[m - 1].imag
                # d/dx (x+iy)^m = m (x+iy)^(m-1); d/dy (x+iy)^m = i m (x+iy)^(m-1)
                G[..., l * l + l + m, 0] = s * q * m * re1
                G[..., l * l + l + m, 1] = -s * q * m * im1
                G[..., l * l + l + m, 2] = s * dq * re
                G[..., l * l + l - m, 0] = s * q * m * im1
                G[..., l * l + l - m, 1] = s * q * m * re1
                G[..., l * l + l - m, 2] = s * dq * im
    if not grad:
        return Y
    # project the polynomial gradient onto the sphere's tangent plane, divide by r
    ug = np.einsum("...k,...lk->...l", u, G)
    G = (G - ug[..., None] * u[..., None, :]) / r[..., None, None]
    return Y, G
