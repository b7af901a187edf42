"""Canonical displacement and neighbour lists (oracle, FP64).

Inclusion rule (the one the HIP library must match bit for bit):

* orthorhombic box (all off-diagonal entries exactly 0): d = x_j - x_i per
  component; in a periodic dimension with edge L, if d > 0.5*L then d -= L,
  else if d < -0.5*L then d += L (positions are kept in [0, L));
* triclinic box H (rows = lattice vectors, r = s H): s = r H^-1 with
  s_k = (x*Hi[0][k] + y*Hi[1][k]) + z*Hi[2][k]; ds = s_j - s_i wrapped at
  +-0.5 the same way; d_k = (ds_0*H[0][k] + ds_1*H[1][k]) + ds_2*H[2][k];
  H^-1 is the cofactor formula below, in this operation order;
* r^2 = (dx*dx + dy*dy) + dz*dz, each operation rounded separately (no fused
  multiply-add); j != i is a neighbour of i iff r^2 < rc*rc.

Lists are full (both i->j and j->i) and sorted by ascending j.
"""
from __future__ import annotations

import numpy as np


def box_inverse(H):
    """Cofactor inverse of a 3x3 box, scalar FP64 operations in a fixed order."""
    H = [[float(H[r][c]) for c in range(3)] for r in range(3)]
    (a, b, c), (d, e, f), (g, h, i) = H
    det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g)
    inv = [
        [(e * i - f * h) / det, (c * h - b * i) / det, (b * f - c * e) / det],
        [(f * g - d * i) / det, (a * i - c * g) / det, (c * d - a * f) / det],
        [(d * h - e * g) / det, (b * g - a * h) / det, (a * e - b * d) / det],
    ]
    return np.array(inv, dtype=np.float64)


def is_orthorhombic(H):
    H = np.asarray(H)
    return bool(np.all(H[~np.eye(3, dtype=bool)] == 0.0))


def perp_widths(H):
    """Perpendicular widths of the cell spanned by the rows of H."""
    H = np.asarray(H, dtype=np.float64)
    vol = abs(np.linalg.det(H))
    return np.array([vol / np.linalg.norm(np.cross(H[(k + 1) % 3], H[(k + 2) % 3])) for k in range(3)])


def frac(pos, Hi):
    """s_k = (x*Hi[0][k] + y*Hi[1][k]) + z*Hi[2][k] (elementwise, no FMA)."""
    x, y, z = pos[..., 0], pos[..., 1], pos[..., 2]
    return np.stack([(x * Hi[0, k] + y * Hi[1, k]) + z * Hi[2, k] for k in range(3)], -1)


def displacement(pos_i, pos_j, H, periodic, Hi=None):
    """Canonical d = r_j - r_i (broadcasting over leading axes)."""
    pos_i = np.asarray(pos_i, dtype=np.float64)
    pos_j = np.asarray(pos_j, dtype=np.float64)
    if is_orthorhombic(H):
        d = pos_j - pos_i
        for k in range(3):
            if periodic[k]:
                L = float(H[k][k])
                half = 0.5 * L
                dk = d[..., k]
                d[..., k] = np.where(dk > half, dk - L, np.where(dk < -half, dk + L, dk))
        return d
    if not all(periodic):
        raise ValueError("triclinic boxes must be periodic in all dimensions")
    if Hi is None:
        Hi = box_inverse(H)
    ds = frac(pos_j, Hi) - frac(pos_i, Hi)
    ds = np.where(ds > 0.5, ds - 1.0, np.where(ds < -0.5, ds + 1.0, ds))
    return np.stack([(ds[..., 0] * H[0][k] + ds[..., 1] * H[1][k]) + ds[..., 2] * H[2][k]
                     for k in range(3)], -1)


def r2_of(d):
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


class Systems:
    """Atoms of one or more independent systems, concatenated."""

    def __init__(self, pos, box, sys_offset, periodic, cutoff):
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.box = np.asarray(box, dtype=np.float64).reshape(-1, 3, 3)
        self.sys_offset = np.asarray(sys_offset, dtype=np.int64)
        self.periodic = tuple(bool(p) for p in periodic)
        self.cutoff = float(cutoff)
        self.rc2 = self.cutoff * self.cutoff
        self.Hi = [box_inverse(H) if not is_orthorhombic(H) else None for H in self.box]
        self.sys_of = np.repeat(np.arange(len(self.box)), np.diff(self.sys_offset))

    @classmethod
    def from_workload(cls, wl, pos=None):
        return cls(wl.pos if pos is None else pos, wl.box, wl.sys_offset, wl.periodic, wl.cutoff)

    @property
    def n_atoms(self):
        return len(self.pos)

    def disp(self, i, js):
        s = self.sys_of[i]
        return displacement(self.pos[i][None, :], self.pos[js], self.box[s], self.periodic, self.Hi[s])

    def neighbours_of(self, i):
        """Brute force over every atom of i's system; returns (j ascending, d)."""
        s = self.sys_of[i]
        lo, hi = self.sys_offset[s], self.sys_offset[s + 1]
        js = np.arange(lo, hi)
        d = self.disp(i, js)
        keep = (r2_of(d) < self.rc2) & (js != i)
        return js[keep], d[keep]

    def neighbour_lists(self, atoms=None):
        """Full lists for the given atoms (default all): list of (j, d)."""
        atoms = range(self.n_atoms) if atoms is None else atoms
        return [self.neighbours_of(int(i)) for i in atoms]

    def neighbour_lists_fast(self):
        """All lists, candidates from a k-d tree on the orthorhombic boxes,
        inclusion decided by the same canonical rule as neighbours_of."""
        from scipy.spatial import cKDTree

        out = [None] * self.n_atoms
        for s in range(len(self.box)):
            lo, hi = int(self.sys_offset[s]), int(self.sys_offset[s + 1])
            H = self.box[s]
            if not is_orthorhombic(H) or hi - lo < 4000:
                for i in range(lo, hi):
                    out[i] = self.neighbours_of(i)
                continue
            p = self.pos[lo:hi].copy()
            size = np.array([H[k][k] if self.periodic[k] else 0.0 for k in range(3)])
            for k in range(3):
                if not self.periodic[k]:
                    p[:, k] -= p[:, k].min()
                    size[k] = p[:, k].max() + 10.0 * self.cutoff
            tree = cKDTree(np.mod(p, size), boxsize=size)
            cand = tree.query_ball_point(np.mod(p, size), self.cutoff * (1 + 1e-6) + 1e-6)
            for ii, c in enumerate(cand):
                i = lo + ii
                js = lo + np.sort(np.asarray(c, dtype=np.int64))
                d = self.disp(i, js)
                keep = (r2_of(d) < self.rc2) & (js != i)
                out[i] = (js[keep], d[keep])
        return out

    def neighbour_finder(self):
        """Callable i -> (j ascending, d) equal to neighbours_of(i): k-d tree
        candidates within the cutoff (plus a margin) on large orthorhombic
        systems, the canonical inclusion rule on every candidate."""
        from scipy.spatial import cKDTree

        trees = {}

        def tree_of(s):
            if s not in trees:
                lo, hi = int(self.sys_offset[s]), int(self.sys_offset[s + 1])
                H = self.box[s]
                if not is_orthorhombic(H) or hi - lo < 4000:
                    trees[s] = None
                else:
                    p = self.pos[lo:hi].copy()
                    shift = np.zeros(3)
                    size = np.array([H[k][k] if self.periodic[k] else 0.0 for k in range(3)])
                    for k in range(3):
                        if not self.periodic[k]:
                            shift[k] = p[:, k].min()
                            size[k] = p[:, k].max() - shift[k] + 10.0 * self.cutoff
                    q = np.mod(p - shift, size)
                    q = np.where(q >= size, 0.0, q)
                    trees[s] = (cKDTree(q, boxsize=size), shift, size, lo)
            return trees[s]

        def find(i):
            s = self.sys_of[i]
            t = tree_of(s)
            if t is None:
                return self.neighbours_of(i)
            tree, shift, size, lo = t
            q = np.mod(self.pos[i] - shift, size)
            q = np.where(q >= size, 0.0, q)
            c = tree.query_ball_point(q, self.cutoff * (1 + 1e-6) + 1e-6)
            js = lo + np.sort(np.asarray(c, dtype=np.int64))
            d = self.disp(i, js)
            keep = (r2_of(d) < self.rc2) & (js != i)
            return js[keep], d[keep]

        return find

    def unique_image_check(self, i):
        """Exactly one periodic image of each neighbour lies within rc."""
        s = self.sys_of[i]
        H = self.box[s]
        js, d = self.neighbours_of(i)
        shifts = np.array([[a, b, c] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                           if all(self.periodic[k] or (a, b, c)[k] == 0 for k in range(3))])
        for j, dj in zip(js, d):
            raw = self.pos[j] - self.pos[i]
            base = np.round(np.linalg.solve(H.T, dj - raw))
            imgs = raw[None, :] + (shifts + base[None, :]) @ H
            n_in = int(np.sum(np.einsum("ik,ik->i", imgs, imgs) < self.rc2))
            if n_in != 1:
                return False
        return True
