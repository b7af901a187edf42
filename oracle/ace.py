"""Atomic cluster expansion for one species (oracle, FP64).

The paper fixes only the energy form E_i = phi_i^(1) + sqrt(phi_i^(2)) with
phi_i^(p) = sum_v c_v^(p) B_iv (section "Atomic cluster expansion"); the
basis itself comes from the cited ACE work and is defined here as follows
(this is the reading both implementations follow):

* radial basis  g_k(r) = T_k(2r/r_c - 1) f_c(r),  f_c = (1 + cos(pi r/r_c))/2,
  k = 0..K-1;  R_nl(r) = sum_k W_nlk g_k(r);
* atomic basis  A_nlm = sum_{j in N(i)} R_nl(r_ij) Y_lm(r_ij / r_ij)
  (real harmonics of ``ylm``);
* coupled pairs AA_{(a,b),L,M} = sum_{m1,m2} C^{l_a l_b L}_{m1 m2 M} A_{a,m1} A_{b,m2}
  (real coupling coefficients of ``cg``), for single indices a=(n_a,l_a) <= b;
* product basis (rows of the model's function list):
  nu=1  B = A_{n00};
  nu=2  B = AA_{(a,b),0,0};
  nu=3  B = sum_M AA_{(a,b),L,M} A_{d,M},         L = l_d;
  nu=4  B = sum_M AA_{(a,b),L,M} AA_{(c,d),L,M};
* embedding  E = phi1 + sqrt(|phi2| + 1e-6): the paper's square-root
  expansion with a guard that keeps it finite for phi2 <= 0; sgn(0) = +1.

Gradients follow the chain rule written out function by function:
dE/dB_v = c1_v + sgn(phi2) c2_v / (2 sqrt(|phi2| + 1e-6)), then the product
rule through each B_v, the coupling sums and finally
dA_nlm/dd_ij = R'_nl(r) (d/r) Y_lm + R_nl dY_lm/dd.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import chebyshev as npcheb

from . import cg as cgmod
from .ylm import real_ylm

EMBED_EPS = 1e-6


class AceOracle:
    def __init__(self, model):
        self.n_max = int(model.n_max)
        self.l_max = int(model.l_max)
        self.K = int(model.K)
        self.r_c = float(model.r_c)
        self.W = np.asarray(model.W, dtype=np.float64)
        self.funcs = np.asarray(model.funcs, dtype=np.int64)
        self.c1 = np.asarray(model.c1, dtype=np.float64)
        self.c2 = np.asarray(model.c2, dtype=np.float64)
        self.nlm = (self.l_max + 1) ** 2
        self.nA = self.n_max * self.nlm
        self._build()

    # ---- index helpers -------------------------------------------------
    def a_index(self, n, l, m):
        """Flat index of A_{n l m}."""
        return n * self.nlm + l * l + l + m

    def _build(self):
        lm1 = self.l_max + 1
        # used coupled-pair channels (a, b, L), a <= b in (n, l) order
        chans = {}

        def chan(n1, l1, n2, l2, L):
            key = (n1 * lm1 + l1, n2 * lm1 + l2, L)
            if key not in chans:
                chans[key] = None
            return key

        for f in self.funcs:
            nu = f[0]
            if nu == 2:
                chan(f[1], f[2], f[3], f[4], 0)
            elif nu == 3:
                chan(f[1], f[2], f[3], f[4], f[9])
            elif nu == 4:
                chan(f[1], f[2], f[3], f[4], f[9])
                chan(f[5], f[6], f[7], f[8], f[9])
        off = 0
        for key in sorted(chans):
            chans[key] = off
            off += 2 * key[2] + 1
        self.chans = chans
        self.nAA = off
        # AA terms: AA[t] += coef * A[i1] * A[i2]
        i1s, i2s, tgt, cof = [], [], [], []
        for (a, b, L), o in chans.items():
            na, la = divmod(a, lm1)
            nb, lb = divmod(b, lm1)
            C = cgmod.cg_real_checked(la, lb, L)
            for m1 in range(-la, la + 1):
                for m2 in range(-lb, lb + 1):
                    for M in range(-L, L + 1):
                        c = C[m1 + la, m2 + lb, M + L]
                        if c != 0.0:
                            i1s.append(self.a_index(na, la, m1))
                            i2s.append(self.a_index(nb, lb, m2))
                            tgt.append(o + M + L)
                            cof.append(c)
        self.aa_i1 = np.asarray(i1s)
        self.aa_i2 = np.asarray(i2s)
        self.aa_coef = np.asarray(cof)
        nt = len(tgt)
        self.S_aa = sp.csr_matrix((np.ones(nt), (np.arange(nt), np.asarray(tgt))), shape=(nt, self.nAA))
        # X = [A (nA) | AA (nAA) | 1]; every B_v = sum_t X[p_t] X[q_t]
        one = self.nA + self.nAA
        self.nX = one + 1
        ps, qs, fs = [], [], []
        for v, f in enumerate(self.funcs):
            nu, L = f[0], f[9]
            if nu == 1:
                ps.append(self.a_index(f[1], 0, 0)); qs.append(one); fs.append(v)
            elif nu == 2:
                o = chans[(f[1] * lm1 + f[2], f[3] * lm1 + f[4], 0)]
                ps.append(self.nA + o); qs.append(one); fs.append(v)
            elif nu == 3:
                o = chans[(f[1] * lm1 + f[2], f[3] * lm1 + f[4], L)]
                for M in range(-L, L + 1):
                    ps.append(self.nA + o + M + L); qs.append(self.a_index(f[5], f[6], M)); fs.append(v)
            elif nu == 4:
                o1 = chans[(f[1] * lm1 + f[2], f[3] * lm1 + f[4], L)]
                o2 = chans[(f[5] * lm1 + f[6], f[7] * lm1 + f[8], L)]
                for M in range(-L, L + 1):
                    ps.append(self.nA + o1 + M + L); qs.append(self.nA + o2 + M + L); fs.append(v)
        self.b_p = np.asarray(ps)
        self.b_q = np.asarray(qs)
        nb = len(fs)
        self.S_b = sp.csr_matrix((np.ones(nb), (np.arange(nb), np.asarray(fs))),
                                 shape=(nb, len(self.funcs)))
        self.S_bT = self.S_b.T.tocsr()
        self.S_p = sp.csr_matrix((np.ones(nb), (np.arange(nb), self.b_p)), shape=(nb, self.nX))
        self.S_q = sp.csr_matrix((np.ones(nb), (np.arange(nb), self.b_q)), shape=(nb, self.nX))
        self.S_i1 = sp.csr_matrix((np.ones(nt), (np.arange(nt), self.aa_i1)), shape=(nt, self.nA))
        self.S_i2 = sp.csr_matrix((np.ones(nt), (np.arange(nt), self.aa_i2)), shape=(nt, self.nA))
        self.n_bterms = nb

    # ---- radial basis ----------------------------------------------------
    def radial(self, r):
        """R[..., n, l] and dR/dr."""
        r = np.asarray(r, dtype=np.float64)
        x = 2.0 * r / self.r_c - 1.0
        fc = 0.5 * (1.0 + np.cos(math.pi * r / self.r_c))
        dfc = -0.5 * math.pi / self.r_c * np.sin(math.pi * r / self.r_c)
        g = np.empty(r.shape + (self.K,))
        dg = np.empty(r.shape + (self.K,))
        for k in range(self.K):
            ck = np.zeros(k + 1)
            ck[k] = 1.0
            T = npcheb.chebval(x, ck)
            dT = npcheb.chebval(x, npcheb.chebder(ck)) if k > 0 else np.zeros_like(x)
            g[..., k] = T * fc
            dg[..., k] = dT * (2.0 / self.r_c) * fc + T * dfc
        R = np.einsum("...k,nlk->...nl", g, self.W)
        dR = np.einsum("...k,nlk->...nl", dg, self.W)
        return R, dR

    # ---- per-atom quantities ------------------------------------------------
    def _lidx(self):
        return np.array([l for l in range(self.l_max + 1) for _ in range(2 * l + 1)])

    def atomic_basis(self, d, mask):
        """A[b, n, lm] for padded bond vectors d[b, j, 3] (mask[b, j] = valid)."""
        dd = np.where(mask[..., None], d, 1.0)
        r = np.sqrt(np.sum(dd * dd, -1))
        R, dR = self.radial(r)
        Y, dY = real_ylm(dd, self.l_max, grad=True)
        li = self._lidx()
        Rl = R[..., li] * mask[..., None, None]           # [b, j, n, lm]
        A = np.einsum("bjnq,bjq->bnq", Rl, Y)
        return A, (r, R, dR, Y, dY, dd)

    def energy_and_grad(self, d_list, batch=None):
        """For each atom (bond vectors d_i[nb, 3]): E_i^ACE and dE_i/dd_ij[nb, 3].

        Also returns phi1, phi2 and the A vector per atom."""
        n = len(d_list)
        E = np.zeros(n)
        phi = np.zeros((n, 2))
        grads = [None] * n
        Aout = np.zeros((n, self.nA))
        if batch is None:
            batch = max(1, int(3e6 // max(1, self.n_bterms)))
        for s in range(0, n, batch):
            idx = list(range(s, min(n, s + batch)))
            nbmax = max(1, max(len(d_list[i]) for i in idx))
            d = np.zeros((len(idx), nbmax, 3))
            mask = np.zeros((len(idx), nbmax), dtype=bool)
            for b, i in enumerate(idx):
                k = len(d_list[i])
                d[b, :k] = d_list[i]
                mask[b, :k] = True
            A3, (r, R, dR, Y, dY, dd) = self.atomic_basis(d, mask)
            A = A3.reshape(len(idx), self.nA)
            AA = (self.S_aa.T @ (A[:, self.aa_i1] * A[:, self.aa_i2] * self.aa_coef).T).T
            X = np.concatenate([A, AA, np.ones((len(idx), 1))], axis=1)
            B = (self.S_bT @ (X[:, self.b_p] * X[:, self.b_q]).T).T
            p1 = B @ self.c1
            p2 = B @ self.c2
            root = np.sqrt(np.abs(p2) + EMBED_EPS)
            Eb = p1 + root
            sgn = np.where(p2 >= 0.0, 1.0, -1.0)
            dEdB = self.c1[None, :] + (sgn / (2.0 * root))[:, None] * self.c2[None, :]
            dterm = (self.S_b @ dEdB.T).T                        # per product term
            dX = (self.S_p.T @ (dterm * X[:, self.b_q]).T).T + (self.S_q.T @ (dterm * X[:, self.b_p]).T).T
            dA = dX[:, : self.nA].copy()
            dAA = dX[:, self.nA: self.nA + self.nAA]
            g = (self.S_aa @ dAA.T).T * self.aa_coef               # dE/dAA at each coupling term
            dA += (self.S_i1.T @ (g * A[:, self.aa_i2]).T).T + (self.S_i2.T @ (g * A[:, self.aa_i1]).T).T
            w = dA.reshape(len(idx), self.n_max, self.nlm)
            li = self._lidx()
            # dE/dd_j = sum_{n,lm} w[n,lm] (dR[j,n,l] Y[j,lm] d/r + R[j,n,l] dY[j,lm,:])
            t1 = np.einsum("bnq,bjnq,bjq->bj", w, dR[..., li], Y)
            t2 = np.einsum("bnq,bjnq,bjqk->bjk", w, R[..., li], dY)
            G = t1[..., None] * dd / r[..., None] + t2
            for b, i in enumerate(idx):
                k = len(d_list[i])
                grads[i] = G[b, :k]
                E[i] = Eb[b]
                phi[i] = (p1[b], p2[b])
                Aout[i] = A[b]
        return E, grads, phi, Aout

    def basis_values(self, d_list):
        """B_v per atom (for invariance pins)."""
        out = []
        for di in d_list:
            d = np.asarray(di)[None]
            mask = np.ones(d.shape[:2], dtype=bool)
            A3, _ = self.atomic_basis(d, mask)
            A = A3.reshape(1, self.nA)
            AA = (self.S_aa.T @ (A[:, self.aa_i1] * A[:, self.aa_i2] * self.aa_coef).T).T
            X = np.concatenate([A, AA, np.ones((1, 1))], axis=1)
            out.append(((self.S_bT @ (X[:, self.b_p] * X[:, self.b_q]).T).T)[0])
        return np.asarray(out)
