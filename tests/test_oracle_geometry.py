"""Pins of the oracle's neighbour search (closed forms and brute force)."""
import math

import numpy as np

from oracle.geometry import Systems, box_inverse, displacement, r2_of
from paper_2505_12958_amd.workloads import lattice_points


def perfect(lattice, n, a, periodic=(True, True, True)):
    p = lattice_points(lattice, (n, n, n), a)
    L = n * a
    return Systems(p, np.diag([L, L, L])[None], [0, len(p)], periodic, 5.5)


def test_bcc_shell_count_58():
    # shells of BCC a=3.165 inside 5.5 A: 8 + 6 + 12 + 24 + 8 = 58
    S = perfect("bcc", 5, 3.165)
    counts = [len(S.neighbours_of(i)[0]) for i in range(0, len(S.pos), 37)]
    assert set(counts) == {58}


def test_fcc_shell_count_54():
    # shells of FCC a=3.615 inside 5.5 A: 12 + 6 + 24 + 12 = 54
    S = perfect("fcc", 4, 3.615)
    counts = [len(S.neighbours_of(i)[0]) for i in range(0, len(S.pos), 29)]
    assert set(counts) == {54}


def test_bcc_first_two_shells_are_14_and_gaps():
    # appendix "Switching function": gaps (1 - sqrt3/2) a and (sqrt2 - 1) a
    a = 3.165
    S = perfect("bcc", 5, a)
    js, d = S.neighbours_of(0)
    r = np.sort(np.sqrt(r2_of(d)))
    assert np.allclose(r[:8], math.sqrt(3) / 2 * a)
    assert np.allclose(r[8:14], a)
    assert np.isclose(r[8] - r[7], (1 - math.sqrt(3) / 2) * a)
    assert np.isclose(r[14] - r[13], (math.sqrt(2) - 1) * a)


def test_lists_sorted_symmetric_and_kdtree_equal():
    rng = np.random.default_rng(3)
    p = lattice_points("bcc", (12, 12, 12), 3.165) + rng.normal(0, 0.08, (3456, 3))
    L = 12 * 3.165
    p[:, :2] = np.mod(p[:, :2], L)
    S = Systems(p, np.diag([L, L, L + 20])[None], [0, len(p)], (True, True, False), 5.5)
    brute = S.neighbour_lists()
    fast = S.neighbour_lists_fast()
    for i in range(len(p)):
        assert np.array_equal(brute[i][0], fast[i][0])
        assert np.all(np.diff(brute[i][0]) > 0)
    # symmetry: j in N(i) <=> i in N(j)
    for i in range(0, len(p), 97):
        for j in brute[i][0]:
            assert i in set(brute[j][0].tolist())


def test_triclinic_unique_image_and_min_image():
    rng = np.random.default_rng(5)
    n, a = 5, 3.165
    e = rng.uniform(-1, 1, 6)
    eps = np.array([[e[0], e[3], e[4]], [e[3], e[1], e[5]], [e[4], e[5], e[2]]])
    eps *= 0.03 / np.max(np.abs(np.linalg.eigvalsh(eps)))
    H = (np.eye(3) * n * a) @ (np.eye(3) + eps)
    frac = lattice_points("bcc", (n, n, n), 1.0) / n
    p = frac @ H + rng.normal(0, 0.08, (len(frac), 3))
    S = Systems(p, H[None], [0, len(p)], (True, True, True), 5.5)
    Hi = box_inverse(H)
    assert np.allclose(Hi @ H, np.eye(3), atol=1e-14)
    for i in range(0, len(p), 7):
        assert S.unique_image_check(i)
    # the canonical displacement is the shortest image for every listed pair
    shifts = np.array([[x, y, z] for x in (-1, 0, 1) for y in (-1, 0, 1) for z in (-1, 0, 1)])
    for i in range(0, len(p), 11):
        js, d = S.neighbours_of(i)
        for j, dj in zip(js, d):
            raw = p[j] - p[i]
            base = np.round(np.linalg.solve(H.T, dj - raw))
            imgs = raw[None] + (shifts + base) @ H
            best = imgs[np.argmin(np.einsum("ik,ik->i", imgs, imgs))]
            assert np.allclose(best, dj, atol=1e-12)


def test_orthorhombic_wrap_rule():
    H = np.diag([10.0, 10.0, 30.0])
    d = displacement(np.array([[0.5, 9.5, 1.0]]), np.array([[9.6, 0.2, 25.0]]), H, (True, True, False))
    assert np.allclose(d, [[-0.9, 0.7, 24.0]])


def test_neighbour_finder_matches_brute_force():
    """The k-d-tree candidate finder returns exactly the brute-force lists
    (same atoms, same displacements) on a slab above its size threshold."""
    from paper_2505_12958_amd import workloads as w

    wl = w.workload(3, scale=13)
    S = Systems.from_workload(wl)
    find = S.neighbour_finder()
    rng = np.random.default_rng(5)
    top = np.argsort(wl.pos[:, 2])[-20:]
    for i in list(rng.choice(wl.n_atoms, 60, replace=False)) + list(top):
        a, da = S.neighbours_of(int(i))
        b, db = find(int(i))
        assert np.array_equal(a, b) and np.array_equal(da, db)
