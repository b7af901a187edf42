"""Seeded synthetic workloads for the adaptive-precision (AP) force path.

This module only *generates inputs*: lattices with jitter, periodic boxes,
Maxwell velocities, fixed/surface masks, the tabulated EAM functions, the
random ACE model (radial mixing weights, basis-function list, expansion
coefficients), the switching rule and the indenter set-up.  It holds none of
the method's energy or force arithmetic; both the HIP library and the FP64
oracle consume what it produces.

Sources for the shapes and numbers (paper: Immel, Mrovec, Drautz, Sutmann,
"Nanoindentation simulations for copper and tungsten with adaptive-precision
potentials", arXiv 2505.12958):

* W EAM analytic form (embedding, pair and density sums, ZBL core and the
  quintic bridge) and its parameter table: appendix "EAM potential" /
  "Optimizing the EAM potential", equations for xi, Phi, zeta_0, zeta,
  xi^Fit, Phi^ZBL, Phi^int, Phi^Fit and the table of optimised parameters.
  The tables built here sample that analytic form; it is the potential
  *definition* (an input), not the AP method.
* Indenter set-up (spherical, cubic potential, moving tip): section
  "Nanoindentation", equation V_ind.
* Switching zones (precise hemisphere under the first-contact point, fast
  surface outside it, CSP-selected atoms elsewhere): section
  "Adaptive-precision potential" and the caption of the set-up figure.
* CSP over the 14 nearest neighbours in BCC: appendix "Switching function".

Units: Angstrom, eV, amu, fs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# physical constants (units: eV, Angstrom, amu, fs)
KB_EV = 8.617333262e-5            # Boltzmann constant, eV/K
ACC = 9.648533212e-3              # (eV/Angstrom/amu) -> Angstrom/fs^2
MASS_W = 183.84
MASS_CU = 63.546
A_W = 3.165                       # lattice constant used by the W-like workloads
A_CU = 3.615                      # lattice constant used by the Cu-like workload
CUTOFF = 5.5
N0_BCC = 58                       # neighbours within 5.5 A of a perfect BCC site (a=3.165)
N0_FCC = 54                       # neighbours within 5.5 A of a perfect FCC site (a=3.615)

# --------------------------------------------------------------------------
# W EAM of the paper's appendix (table of optimised parameters at 300 K)
W_EAM = dict(
    r_lo=1.10002200044, r_hi=2.10004200084, Z=74.0, eps0=0.005526349406,
    a_zbl=0.08702457248897934,
    a_phi=[3663.54, -3663.85, 128.443, 2.10845, 5.10311, -4.06894, 1.25081,
           1.64931, -1.4248, -0.761194, 1.93524, -0.70151, 0.0935973,
           -1.40395, 1.13035],
    d_phi=[2.74456, 2.74451, 2.28653, 2.91147, 2.96512, 3.07694, 3.53116,
           3.85904, 4.10323, 4.73354, 4.8959, 5.09081, 5.27739, 5.40309,
           5.45078],
    a_rho=[-267.394, 0.486763, -0.0425619, 0.0330214],
    d_rho=[2.5, 3.1, 3.5, 4.9],
    a_xi=[-6.24657, -0.0836583], d_xi=-2.14333,
    b_phi=[15390.7852469191, -41436.4792651818, 45168.4307517119,
           -24693.6420961014, 6736.28696027297, -731.611626209140],
    r_cut_rho=2.46396652011306,
)
ZBL_C = [(0.1818, 3.2), (0.5099, 0.9423), (0.2802, 0.4029), (0.02817, 0.2016)]


def _knot_sum(r, a, d):
    """sum_i a_i (d_i - r)^3 Theta(d_i - r) and its r-derivative."""
    r = np.asarray(r, dtype=np.float64)
    v = np.zeros_like(r)
    dv = np.zeros_like(r)
    for ai, di in zip(a, d):
        t = np.where(di - r >= 0.0, di - r, 0.0)
        v += ai * t ** 3
        dv += -3.0 * ai * t ** 2
    return v, dv


def w_pair(r):
    """Phi^Fit(r): ZBL below r_lo, quintic bridge on [r_lo, r_hi], knot sum above."""
    p = W_EAM
    r = np.asarray(r, dtype=np.float64)
    pref = p["Z"] * p["Z"] / (4.0 * math.pi * p["eps0"])
    x = r / p["a_zbl"]
    scr = sum(c * np.exp(-k * x) for c, k in ZBL_C)
    dscr = sum(-c * k / p["a_zbl"] * np.exp(-k * x) for c, k in ZBL_C)
    zbl = pref * scr / r
    dzbl = pref * (dscr / r - scr / r ** 2)
    poly = sum(b * r ** m for m, b in enumerate(p["b_phi"]))
    dpoly = sum(m * b * r ** (m - 1) for m, b in enumerate(p["b_phi"]) if m > 0)
    knot, dknot = _knot_sum(r, p["a_phi"], p["d_phi"])
    v = np.where(r < p["r_lo"], zbl, np.where(r <= p["r_hi"], poly, knot))
    dv = np.where(r < p["r_lo"], dzbl, np.where(r <= p["r_hi"], dpoly, dknot))
    return v, dv


def w_density(r):
    """zeta(r): zeta_0 held at its maximum value below r_cut^rho."""
    p = W_EAM
    r = np.asarray(r, dtype=np.float64)
    z0, dz0 = _knot_sum(r, p["a_rho"], p["d_rho"])
    zc, _ = _knot_sum(np.array([p["r_cut_rho"]]), p["a_rho"], p["d_rho"])
    v = np.where(r <= p["r_cut_rho"], zc[0], z0)
    dv = np.where(r <= p["r_cut_rho"], 0.0, dz0)
    return v, dv


def w_embed(rho):
    """xi^Fit(rho) = a1 sqrt(rho) + a2 rho^2 + Delta xi."""
    p = W_EAM
    rho = np.asarray(rho, dtype=np.float64)
    a1, a2 = p["a_xi"]
    s = np.sqrt(np.maximum(rho, 0.0))
    v = a1 * s + a2 * rho ** 2 + p["d_xi"]
    with np.errstate(divide="ignore"):
        dv = np.where(rho > 0, 0.5 * a1 / np.where(rho > 0, s, 1.0), -np.inf) + 2 * a2 * rho
    return v, dv


# --------------------------------------------------------------------------
# tables: uniform knots, piecewise cubic stored as coef[k] = (c0, c1, c2, c3)
@dataclass
class Table:
    x0: float
    dx: float
    n_knots: int
    coef: np.ndarray          # (n_knots-1, 4) float64, value = c0 + c1 t + c2 t^2 + c3 t^3

    def arrays(self):
        return dict(x0=self.x0, dx=self.dx, n_knots=self.n_knots, coef=self.coef)


def _smooth_noise(rng, n, amp):
    """Seeded smooth multiplicative noise on n knots, zero at both ends."""
    if amp == 0.0:
        return np.zeros(n)
    u = np.linspace(0.0, 1.0, n)
    xi = np.zeros(n)
    for k in range(1, 7):
        xi += rng.normal() * np.sin(k * math.pi * u + rng.uniform(0, 2 * math.pi)) / k
    xi *= np.sin(math.pi * u)
    xi /= max(1e-12, np.max(np.abs(xi)))
    return amp * xi


def spline_table(f, x0, x1, n_knots, left, right, rng=None, noise=0.0):
    """Clamped (or natural) cubic spline through f at uniform knots.

    left/right: ('slope', value) or ('natural',).  Returns a Table whose
    piecewise cubic *is* the tabulated function seen by both the library and
    the oracle.
    """
    from scipy.interpolate import CubicSpline

    x = x0 + (x1 - x0) * np.arange(n_knots) / (n_knots - 1)
    y = np.asarray(f(x), dtype=np.float64)
    if noise:
        y = y * (1.0 + _smooth_noise(rng, n_knots, noise))

    def bc(spec):
        return "natural" if spec[0] == "natural" else (1, float(spec[1]))

    cs = CubicSpline(x, y, bc_type=(bc(left), bc(right)))
    coef = np.ascontiguousarray(cs.c[::-1].T)          # (n-1, 4): c0..c3
    return Table(x0=float(x0), dx=float((x1 - x0) / (n_knots - 1)), n_knots=n_knots, coef=coef)


def _perfect_density(a, lattice, scale):
    """Host-density of a perfect-lattice site from the analytic zeta (setup only)."""
    basis = _basis(lattice)
    n = 4
    pts = []
    for i in range(-n, n + 1):
        for j in range(-n, n + 1):
            for k in range(-n, n + 1):
                for b in basis:
                    pts.append((np.array([i, j, k]) + b) * a)
    pts = np.array(pts)
    r = np.linalg.norm(pts, axis=1)
    r = r[(r > 1e-9) & (r < CUTOFF)]
    return float(np.sum(w_density(r * scale)[0]))


@dataclass
class EamTables:
    phi: Table
    rho: Table
    F: Table


def make_eam_tables(kind="W", n_knots=500, noise=0.01, seed=0, r_min=1.0, r_c=CUTOFF):
    """W-like (kind='W') or Cu-like (kind='Cu') tables sampled from the W EAM.

    Cu-like tables stretch r by the nearest-neighbour ratio W/Cu so the first
    shell of FCC a=3.615 maps onto the first shell of BCC a=3.165.  noise
    multiplies the knot values by (1 + noise*xi_k) with smooth seeded xi_k
    tapered to zero at both ends; noise=0 gives the paper's W EAM.
    """
    rng = np.random.default_rng(seed)
    if kind == "W":
        scale = 1.0
        lattice, a = "bcc", 3.1837
    elif kind == "Cu":
        scale = (A_W * math.sqrt(3) / 2) / (A_CU / math.sqrt(2))
        lattice, a = "fcc", A_CU
    else:
        raise ValueError(kind)

    def phi(r):
        return w_pair(r * scale)[0]

    def dens(r):
        return w_density(r * scale)[0]

    t_phi = spline_table(phi, r_min, r_c, n_knots, ("slope", w_pair(r_min * scale)[1] * scale),
                         ("slope", 0.0), rng, noise)
    t_rho = spline_table(dens, r_min, r_c, n_knots, ("slope", w_density(r_min * scale)[1] * scale),
                         ("slope", 0.0), rng, noise)
    rho_b = _perfect_density(a, lattice, scale)
    rho_max = 2.0 * rho_b
    t_F = spline_table(lambda x: w_embed(x)[0], 0.0, rho_max, n_knots, ("natural",),
                       ("slope", w_embed(np.array([rho_max]))[1][0]), rng, noise)
    return EamTables(phi=t_phi, rho=t_rho, F=t_F)


# --------------------------------------------------------------------------
# ACE model: radial mixing weights, basis list, two coefficient sets
@dataclass
class AceModel:
    n_max: int
    l_max: int
    nu_max: int
    K: int
    r_c: float
    W: np.ndarray              # (n_max, l_max+1, K) float64
    funcs: np.ndarray          # (n_funcs, 10) int32: nu, n1,l1, n2,l2, n3,l3, n4,l4, L
    c1: np.ndarray             # (n_funcs,) float64
    c2: np.ndarray             # (n_funcs,) float64


def _coupling_ok(l1, l2, L):
    return abs(l1 - l2) <= L <= l1 + l2 and (l1 + l2 + L) % 2 == 0


def enumerate_basis(n_max, l_max, nu_max):
    """Canonical non-redundant product-basis list of the model file.

    Single-index (n,l) pairs are ordered by n, then l.  nu=1: A_{n00};
    nu=2: pairs a<=b of equal l coupled to L=0; nu=3: sorted triples a<=b<=d
    with (a,b) coupled to L=l_d; nu=4: sorted quadruples a<=b<=c<=d with
    (a,b) and (c,d) each coupled to a common L.  Only couplings with
    l1+l2+L even are kept (their real-basis coupling coefficients are real).
    Rows: nu, n1,l1, n2,l2, n3,l3, n4,l4, L (unused slots are -1).
    """
    idx = [(n, l) for n in range(n_max) for l in range(l_max + 1)]
    A = len(idx)
    rows = []
    for a in range(A):
        if idx[a][1] == 0:
            rows.append([1, *idx[a], -1, -1, -1, -1, -1, -1, 0])
    if nu_max >= 2:
        for a in range(A):
            for b in range(a, A):
                if idx[a][1] == idx[b][1]:
                    rows.append([2, *idx[a], *idx[b], -1, -1, -1, -1, 0])
    if nu_max >= 3:
        for a in range(A):
            for b in range(a, A):
                for d in range(b, A):
                    if _coupling_ok(idx[a][1], idx[b][1], idx[d][1]):
                        rows.append([3, *idx[a], *idx[b], *idx[d], -1, -1, idx[d][1]])
    if nu_max >= 4:
        for a in range(A):
            for b in range(a, A):
                for c in range(b, A):
                    for d in range(c, A):
                        la, lb, lc, ld = idx[a][1], idx[b][1], idx[c][1], idx[d][1]
                        for L in range(0, 2 * l_max + 1):
                            if _coupling_ok(la, lb, L) and _coupling_ok(lc, ld, L):
                                rows.append([4, *idx[a], *idx[b], *idx[c], *idx[d], L])
    if nu_max >= 5:
        raise ValueError("nu_max <= 4 supported")
    return np.asarray(rows, dtype=np.int32).reshape(-1, 10)


def make_ace_model(n_max, l_max, nu_max, seed, n0, r_c=CUTOFF, coef_std=0.1):
    ss = np.random.SeedSequence(seed).spawn(3)
    K = n_max
    W = np.random.default_rng(ss[0]).standard_normal((n_max, l_max + 1, K)) / (math.sqrt(K) * n0)
    funcs = enumerate_basis(n_max, l_max, nu_max)
    c1 = np.random.default_rng(ss[1]).normal(0.0, coef_std, len(funcs))
    c2 = np.random.default_rng(ss[2]).normal(0.0, coef_std, len(funcs))
    return AceModel(n_max, l_max, nu_max, K, float(r_c), W, funcs, c1, c2)


# --------------------------------------------------------------------------
# lattices and systems
def _basis(lattice):
    if lattice == "bcc":
        return [np.zeros(3), np.array([0.5, 0.5, 0.5])]
    if lattice == "fcc":
        return [np.zeros(3), np.array([0.5, 0.5, 0.0]), np.array([0.5, 0.0, 0.5]),
                np.array([0.0, 0.5, 0.5])]
    raise ValueError(lattice)


def lattice_points(lattice, n, a):
    """Perfect lattice of n[0] x n[1] x n[2] cubic cells; row-major cell order."""
    basis = np.array(_basis(lattice))
    g = np.stack(np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij"), -1)
    g = g.reshape(-1, 1, 3) + basis[None, :, :]
    return (g.reshape(-1, 3) * a).astype(np.float64)


@dataclass
class LambdaRule:
    kind: int                     # 0 const, 1 sphere, 2 hemisphere, 3 mask (+ hemisphere)
    value: float = 0.0
    centre: tuple = (0.0, 0.0, 0.0)
    r_full: float = 0.0
    taper: float = 0.0
    z_surface_min: float = float("inf")
    mask: np.ndarray | None = None   # uint8 per atom (kind 3)


LAMBDA_CONST, LAMBDA_SPHERE, LAMBDA_HEMISPHERE, LAMBDA_MASK = 0, 1, 2, 3


@dataclass
class Workload:
    name: str
    pos: np.ndarray               # (N, 3) float64
    box: np.ndarray               # (n_sys, 3, 3) float64, rows = lattice vectors
    sys_offset: np.ndarray        # (n_sys+1,) int64
    periodic: tuple
    cutoff: float
    masses: np.ndarray            # (N,) float64
    fixed: np.ndarray             # (N,) uint8
    vel: np.ndarray               # (N, 3) float64
    eam: EamTables | None
    ace: AceModel | None
    rule: LambdaRule
    indenter: dict = field(default_factory=dict)   # centre, vel, R, K (K<=0: none)
    dt: float = 2.0
    steps: int = 0
    meta: dict = field(default_factory=dict)
    nvt: np.ndarray | None = None  # (N,) bool: Nose-Hoover layer (None: none)

    @property
    def n_atoms(self):
        return len(self.pos)

    @property
    def n_systems(self):
        return len(self.box)


def maxwell(rng, masses, mobile, T):
    v = rng.standard_normal((len(masses), 3)) * np.sqrt(KB_EV * T * ACC / masses)[:, None]
    v[~mobile] = 0.0
    nm = int(mobile.sum())
    if nm > 1:
        p = (masses[mobile, None] * v[mobile]).sum(0) / masses[mobile].sum()
        v[mobile] -= p
        ke = 0.5 * np.sum(masses[mobile, None] * v[mobile] ** 2) / ACC
        dof = 3 * nm - 3
        v[mobile] *= math.sqrt(T / (2.0 * ke / (dof * KB_EV)))
    return v


def csp_values(pos, box_lengths, periodic, n_nb=14):
    """Centro-symmetry parameter: sum of the n_nb/2 smallest |d_a + d_b|^2
    pair sums over the n_nb nearest neighbours (setup-time mask only)."""
    from scipy.spatial import cKDTree

    size = np.array([L if p else 1e9 for L, p in zip(box_lengths, periodic)])
    p = pos.copy()
    for k in range(3):
        if periodic[k]:
            p[:, k] = np.mod(p[:, k], size[k])
        else:
            p[:, k] = p[:, k] - p[:, k].min() + 1.0
    tree = cKDTree(p, boxsize=size)
    _, nb = tree.query(p, k=n_nb + 1)
    nb = nb[:, 1:]
    d = p[nb] - p[:, None, :]
    for k in range(3):
        if periodic[k]:
            d[..., k] -= size[k] * np.round(d[..., k] / size[k])
    ia, ib = np.triu_indices(n_nb, 1)
    s = d[:, ia, :] + d[:, ib, :]
    s2 = np.sort(np.einsum("npk,npk->np", s, s), axis=1)
    return s2[:, : n_nb // 2].sum(1)


def _rule_geom(pos, centre, r_full, taper):
    """Geometric part of the switching rule, used only to size the mask."""
    d = np.linalg.norm(pos - np.asarray(centre)[None, :], axis=1)
    return d <= r_full + taper


def make_slab(name, lattice, ncell, a, kind, seed, *, n_max, l_max, nu_max, n0, mass,
              r_full=30.0, taper=5.0, jitter=0.05, ace_frac=None, indent_depth=0.5,
              indent_speed=5e-5, static_indent=None, R=40.0, K=10.0, T=300.0, dt=2.0,
              steps=200, vacuum=30.0):
    """Free-top slab periodic in x/y with 3 fixed unit-cell layers at the bottom.

    Indenter: spherical tip of radius R above the centre of the top surface,
    first contact at depth indent_depth below the top plane, moving down at
    indent_speed (A/fs); static_indent=h puts it at depth h (atoms inside the
    tip removed) with zero speed.
    """
    ss = np.random.SeedSequence(seed).spawn(8)
    pos = lattice_points(lattice, ncell, a)
    Lx, Ly = ncell[0] * a, ncell[1] * a
    z_top = pos[:, 2].max()
    centre_surface = np.array([Lx / 2, Ly / 2, z_top])
    if static_indent is not None:
        tip = np.array([Lx / 2, Ly / 2, z_top + R - static_indent])
        keep = np.linalg.norm(pos - tip[None, :], axis=1) >= R
        pos = pos[keep]
        ind = dict(centre=tip, vel=np.zeros(3), R=R, K=K)
    else:
        tip = np.array([Lx / 2, Ly / 2, z_top + R - indent_depth])
        ind = dict(centre=tip, vel=np.array([0.0, 0.0, -indent_speed]), R=R, K=K)
    n = len(pos)
    pos = pos + np.random.default_rng(ss[0]).normal(0.0, jitter, pos.shape)
    pos[:, 0] = np.mod(pos[:, 0], Lx)
    pos[:, 1] = np.mod(pos[:, 1], Ly)
    Lz = ncell[2] * a + vacuum
    box = np.diag([Lx, Ly, Lz])[None].astype(np.float64)
    fixed = (pos[:, 2] < 3 * a - a / 4).astype(np.uint8)
    z_surf = (ncell[2] - 1) * a - a / 4
    masses = np.full(n, mass)
    vel = maxwell(np.random.default_rng(ss[1]), masses, fixed == 0, T)
    eam = make_eam_tables(kind, noise=0.01, seed=int(ss[2].generate_state(1)[0]))
    ace = make_ace_model(n_max, l_max, nu_max, int(ss[3].generate_state(1)[0]), n0)
    if ace_frac is None:
        rule = LambdaRule(LAMBDA_HEMISPHERE, centre=tuple(centre_surface), r_full=r_full,
                          taper=taper, z_surface_min=z_surf)
    else:
        csp = csp_values(pos, (Lx, Ly, Lz), (True, True, False))
        geo = _rule_geom(pos, centre_surface, r_full, taper)
        interior = (fixed == 0) & (pos[:, 2] < z_surf) & ~geo
        need = max(0, int(round(ace_frac * n)) - int(geo.sum()))
        vals = np.sort(csp[interior])[::-1]
        theta = vals[min(need, len(vals)) - 1] if need > 0 else np.inf
        mask = (interior & (csp >= theta)).astype(np.uint8)
        rule = LambdaRule(LAMBDA_MASK, centre=tuple(centre_surface), r_full=r_full, taper=taper,
                          z_surface_min=z_surf, mask=mask)
    return Workload(name=name, pos=pos, box=box, sys_offset=np.array([0, n], np.int64),
                    periodic=(True, True, False), cutoff=CUTOFF, masses=masses, fixed=fixed,
                    vel=vel, eam=eam, ace=ace, rule=rule, indenter=ind, dt=dt, steps=steps,
                    meta=dict(z_top=z_top, lattice=lattice, a=a, ncell=tuple(ncell)))


# The paper's nanoindentation set-ups (tables of simulation parameters for
# W and Cu in section "Results"; thermostat time constant from step 4 of the
# equilibration table).  Lengths A, times fs, velocities A/fs
# (20 m/s = 2e-4 A/fs), k_ind eV/A^3.
INDENT_W = dict(lattice="bcc", a=A_W, mass=MASS_W, n_cells=86, T=300.0, h_fixed=20.0, h_nvt=10.0,
                dt=1.0, R=60.0, speed=2.0e-4, K=236.0, h_max=20.8, h0=-4.2, tau=100.0)
W_EAM_A0 = 3.1837                 # lattice constant of the paper's W EAM (properties table, EAM fit)
INDENT_CU = dict(lattice="fcc", a=A_CU, mass=MASS_CU, n_cells=100, T=292.0, h_fixed=10.0,
                 h_nvt=10.0, dt=1.0, R=60.0, speed=2.5e-4, K=10.0, h_max=20.0, h0=-5.0, tau=100.0)


def make_indentation(setup, *, n_cells=None, a=None, seed=7, vacuum=30.0, eam=None, ace=None,
                     rule=None):
    """Slab of the paper's nanoindentation set-up: an (100) surface on top,
    periodic in x and y, the bottom h_fixed A fixed, the next h_nvt A the
    Nose-Hoover layer, the rest NVE; Maxwell velocities at T on the mobile
    atoms; the spherical indenter above the centre of the surface with its
    lowest point h0 above the top atomic plane, moving down at `speed`.
    n_cells (default: the paper's box, 86 cells of W = 1,272,112 atoms, 100
    cells of Cu = 4,000,000 atoms) sets the cube edge in unit cells; a
    (default the set-up's) is the lattice constant, which should be the
    potential's own so that the slab starts at its equilibrium density.  The
    potential (eam, ace, rule) is the caller's; rule defaults to lambda = 0
    (EAM everywhere)."""
    p = setup
    n = p["n_cells"] if n_cells is None else n_cells
    a = p["a"] if a is None else float(a)
    pos = lattice_points(p["lattice"], (n, n, n), a)
    N = len(pos)
    L = n * a
    z_top = float(pos[:, 2].max())
    z0 = float(pos[:, 2].min())
    fixed = (pos[:, 2] < z0 + p["h_fixed"]).astype(np.uint8)
    nvt = (fixed == 0) & (pos[:, 2] < z0 + p["h_fixed"] + p["h_nvt"])
    masses = np.full(N, p["mass"])
    vel = maxwell(np.random.default_rng(seed), masses, fixed == 0, p["T"])
    centre = np.array([L / 2, L / 2, z_top + p["R"] - p["h0"]])
    ind = dict(centre=centre, vel=np.array([0.0, 0.0, -p["speed"]]), R=p["R"], K=p["K"])
    box = np.diag([L, L, n * a + vacuum + p["R"]])[None].astype(np.float64)
    if rule is None:
        rule = LambdaRule(LAMBDA_CONST, value=0.0)
    return Workload(name=f"indent-{p['lattice']}-{n}", pos=pos, box=box,
                    sys_offset=np.array([0, N], np.int64), periodic=(True, True, False),
                    cutoff=CUTOFF, masses=masses, fixed=fixed, vel=vel, eam=eam, ace=ace, rule=rule,
                    indenter=ind, dt=p["dt"], steps=0, nvt=nvt,
                    meta=dict(z_top=z_top, lattice=p["lattice"], a=a, ncell=(n, n, n),
                              setup=dict(p, a=a)))


def make_crystal(lattice, ncell, a, mass, T, seed=0):
    """Perfect fully periodic cube of ncell^3 unit cells with Maxwell
    velocities at T; lambda = 0 everywhere, no potential attached."""
    pos = lattice_points(lattice, (ncell,) * 3, a)
    n = len(pos)
    L = ncell * a
    masses = np.full(n, mass)
    vel = maxwell(np.random.default_rng(seed), masses, np.ones(n, bool), T)
    return Workload(name=f"{lattice}-crystal-{ncell}", pos=pos,
                    box=np.diag([L, L, L])[None].astype(np.float64),
                    sys_offset=np.array([0, n], np.int64), periodic=(True, True, True),
                    cutoff=CUTOFF, masses=masses, fixed=np.zeros(n, np.uint8), vel=vel, eam=None,
                    ace=None, rule=LambdaRule(LAMBDA_CONST, value=0.0), indenter=dict(K=0.0), dt=1.0,
                    steps=0, meta=dict(lattice=lattice, a=a, ncell=(ncell,) * 3))


def make_bulk(name, ncell, a, seed, *, n_max, l_max, nu_max, jitter=0.05, r_full=10.0,
              taper=5.0, kind="W"):
    """Fully periodic BCC cube with a spherical precise region at its centre."""
    ss = np.random.SeedSequence(seed).spawn(8)
    pos = lattice_points("bcc", (ncell,) * 3, a)
    L = ncell * a
    pos = np.mod(pos + np.random.default_rng(ss[0]).normal(0.0, jitter, pos.shape), L)
    n = len(pos)
    masses = np.full(n, MASS_W)
    vel = maxwell(np.random.default_rng(ss[1]), masses, np.ones(n, bool), 300.0)
    eam = make_eam_tables(kind, noise=0.01, seed=int(ss[2].generate_state(1)[0]))
    ace = make_ace_model(n_max, l_max, nu_max, int(ss[3].generate_state(1)[0]), N0_BCC)
    rule = LambdaRule(LAMBDA_SPHERE, centre=(L / 2, L / 2, L / 2), r_full=r_full, taper=taper)
    return Workload(name=name, pos=pos, box=np.diag([L, L, L])[None].astype(np.float64),
                    sys_offset=np.array([0, n], np.int64), periodic=(True, True, True),
                    cutoff=CUTOFF, masses=masses, fixed=np.zeros(n, np.uint8), vel=vel, eam=eam,
                    ace=ace, rule=rule, indenter=dict(K=0.0), dt=1.0, steps=0,
                    meta=dict(lattice="bcc", a=a, ncell=(ncell,) * 3))


def make_batch(name, n_cells, seed, *, n_min=250, n_maxatoms=16000, strain_max=0.03,
               jitter=0.08, a=A_W, n_max=6, l_max=3, nu_max=3):
    """Independent periodic BCC cells under random homogeneous strain (triclinic)."""
    ss = np.random.SeedSequence(seed).spawn(8)
    rs = np.random.default_rng(ss[0])
    sizes = np.exp(rs.uniform(math.log(n_min), math.log(n_maxatoms), n_cells))
    nc = np.clip(np.round(np.cbrt(sizes / 2.0)).astype(int), 5, 20)
    rj = np.random.default_rng(ss[1])
    rstr = np.random.default_rng(ss[2])
    pos_all, boxes, offs = [], [], [0]
    for c in range(n_cells):
        n = int(nc[c])
        e6 = rstr.uniform(-1, 1, 6)
        eps = np.array([[e6[0], e6[3], e6[4]], [e6[3], e6[1], e6[5]], [e6[4], e6[5], e6[2]]])
        eps *= rstr.uniform(0.0, strain_max) / np.max(np.abs(np.linalg.eigvalsh(eps)))
        H0 = np.eye(3) * n * a
        H = H0 @ (np.eye(3) + eps)                  # rows are lattice vectors
        frac = lattice_points("bcc", (n, n, n), 1.0) / n
        p = frac @ H + rj.normal(0.0, jitter, (len(frac), 3))
        pos_all.append(p)
        boxes.append(H)
        offs.append(offs[-1] + len(p))
    pos = np.concatenate(pos_all)
    N = len(pos)
    ace = make_ace_model(n_max, l_max, nu_max, int(ss[3].generate_state(1)[0]), N0_BCC)
    eam = make_eam_tables("W", noise=0.01, seed=int(ss[4].generate_state(1)[0]))
    return Workload(name=name, pos=pos, box=np.asarray(boxes), sys_offset=np.asarray(offs, np.int64),
                    periodic=(True, True, True), cutoff=CUTOFF, masses=np.full(N, MASS_W),
                    fixed=np.zeros(N, np.uint8), vel=np.zeros((N, 3)), eam=eam, ace=ace,
                    rule=LambdaRule(LAMBDA_CONST, value=1.0), indenter=dict(K=0.0), dt=1.0,
                    steps=0, meta=dict(cells=nc.tolist()))


def workload(k, *, scale=None, seed=None):
    """The five standard workloads (k = 1..5), seed = 1000 + k by default.

    scale shrinks the slab / batch for oracle-sized parity runs while keeping
    the structure (same lattice, boundaries, switching rule and ACE model size).
    """
    seed = 1000 + k if seed is None else seed
    if k == 1:
        n = 10 if scale is None else scale
        return make_bulk("bcc-w-bulk-2000", n, A_W, seed, n_max=6, l_max=3, nu_max=3)
    if k == 2:
        n = 30 if scale is None else scale
        return make_slab(f"fcc-cu-slab-{n}", "fcc", (n, n, n), A_CU, "Cu", seed, n_max=6, l_max=3,
                         nu_max=3, n0=N0_FCC, mass=MASS_CU,
                         r_full=30.0 if scale is None else min(30.0, n * A_CU / 4),
                         steps=200)
    if k == 3:
        n = 50 if scale is None else scale
        return make_slab(f"bcc-w-slab-{n}", "bcc", (n, n, n), A_W, "W", seed, n_max=8, l_max=4,
                         nu_max=4, n0=N0_BCC, mass=MASS_W, ace_frac=0.08,
                         r_full=30.0 if scale is None else min(30.0, n * A_W / 4),
                         steps=200)
    if k == 4:
        cells = 96 if scale is None else scale
        return make_batch(f"bcc-w-batch-{cells}", cells, seed,
                          n_maxatoms=16000 if scale is None else 2000)
    if k == 5:
        n = 110 if scale is None else scale
        return make_slab(f"bcc-w-slab-{n}-static", "bcc", (n, n, n), A_W, "W", seed, n_max=8,
                         l_max=4, nu_max=4, n0=N0_BCC, mass=MASS_W,
                         r_full=60.0 if scale is None else min(60.0, n * A_W / 4),
                         static_indent=15.0, steps=100)
    raise ValueError(k)
