"""Finite-difference checks through the C ABI on the full 250,000-atom W slab
(nu <= 4 ACE region of 20,000 atoms, indenter in contact): the forces of the
FP64 and mixed paths on 64 sampled atoms against central differences (one
Richardson step) of the FP64 GPU energy at fixed lambda.

Moving one atom changes only the per-atom energies of the atoms within the
cutoff of it (and the indenter energy), so each difference is taken over the
per-atom energies of the atoms within r_c + 0.5 A of the moved atom; their
ACE energies come from the same kernels with the ACE list restricted to
them.  This keeps the rounding noise of a 250k-term sum out of the
differences.  Atoms whose |phi2| < 1e-4 sit on the kink of the embedding
guard and are not sampled."""
import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

from oracle.ap import APOracle
from oracle.geometry import Systems
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu


class LocalEnergy:
    """FP64 GPU energy of the atoms near a moved atom, lambda fixed."""

    def __init__(self, wl, lam):
        self.wl = wl
        self.ctx = ap.Context(wl.eam, wl.ace, ap.AP_PREC_FP64)
        self.S = ap.SystemsArg.from_workload(wl)
        N = wl.n_atoms
        self.nl = ap.NeighbourList(N, 64)
        self.lam = torch.tensor(lam, dtype=torch.float64, device="cuda")
        self.is_ace = lam > 0
        self.acl = torch.zeros(N, dtype=torch.int32, device="cuda")
        self.nac = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.e_atom = torch.zeros(N, dtype=torch.float64, device="cuda")
        self.F = torch.zeros((3, N), dtype=torch.float64, device="cuda")
        self.e_ind = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.fixed = torch.tensor(wl.fixed, dtype=torch.uint8, device="cuda")
        size = np.array([wl.box[0][k][k] if wl.periodic[k] else 1e9 for k in range(3)])
        p = wl.pos.copy()
        p[:, 2] -= p[:, 2].min()
        self.tree = cKDTree(np.mod(p, size), boxsize=size)
        self.size = size
        self.zmin = wl.pos[:, 2].min()

    def near(self, i):
        q = self.wl.pos[i].copy()
        q[2] -= self.zmin
        return np.sort(np.asarray(self.tree.query_ball_point(np.mod(q, self.size), self.wl.cutoff + 0.5)))

    def __call__(self, pos, local):
        ind = self.wl.indenter
        loc_ace = local[self.is_ace[local]].astype(np.int32)
        self.acl[: len(loc_ace)] = torch.tensor(loc_ace, device="cuda")
        self.nac.fill_(len(loc_ace))
        P = torch.tensor(np.ascontiguousarray(pos.T), dtype=torch.float64, device="cuda")
        self.ctx.build_neighbors(self.S, P, self.nl)
        self.ctx.eam_forces(self.S, P, self.nl, self.lam, self.e_atom, self.F)
        self.ctx.ace_forces(self.S, P, self.nl, self.lam, self.acl, self.nac, self.e_atom, self.F,
                            accumulate=True)
        self.ctx.indenter(self.S, P, self.fixed, ind["centre"], ind["R"], ind["K"], self.F,
                          e_ind=self.e_ind)
        e = self.e_atom[torch.tensor(local, device="cuda")].cpu().numpy()
        return float(np.sum(e)) + float(self.e_ind.item())


def forces(wl, precision):
    ctx = ap.Context(wl.eam, wl.ace, precision)
    st = ap.MD(wl)
    ctx.step(st.sys, st, 0)
    torch.cuda.synchronize()
    ctx.check()
    out = st.force.cpu().numpy().T.copy(), st.lam.cpu().numpy()
    ctx.close()
    return out


def test_forces_match_fd_of_fp64_energy_full_slab():
    wl = w.workload(3)
    F64, lam = forces(wl, ap.AP_PREC_FP64)
    Fmx, _ = forces(wl, ap.AP_PREC_MIXED)
    rng = np.random.default_rng(3)
    ace = rng.permutation(np.nonzero(lam > 0)[0])[:80]
    S = Systems.from_workload(wl)
    find = S.neighbour_finder()
    nl = {int(i): find(int(i)) for i in ace}
    _, _, _, _, phi = APOracle(None, wl.ace).bond_terms(S, lam, [int(i) for i in ace], nl)
    ace = [int(i) for i, ph in zip(ace, phi) if abs(ph[1]) >= 1e-4][:48]
    # EAM-only atoms, a few of them under the tip
    eam = np.nonzero(lam == 0)[0]
    d_tip = np.linalg.norm(wl.pos[eam] - wl.indenter["centre"][None, :], axis=1)
    touch = eam[d_tip < wl.indenter["R"]]
    pick = list(rng.choice(touch, min(4, len(touch)), replace=False)) if len(touch) else []
    pick += list(rng.choice(eam, 64 - len(ace) - len(pick), replace=False))
    atoms = ace + [int(i) for i in pick]
    E = LocalEnergy(wl, lam)
    h = 2e-4
    fd = np.zeros((len(atoms), 3))
    for t, i in enumerate(atoms):
        local = E.near(i)
        for k in range(3):
            def d(hh):
                p = wl.pos.copy(); p[i, k] += hh
                m = wl.pos.copy(); m[i, k] -= hh
                return (E(p, local) - E(m, local)) / (2 * hh)
            fd[t, k] = -(4 * d(h / 2) - d(h)) / 3
    E.ctx.close()
    scale = np.linalg.norm(fd)
    e64 = np.linalg.norm(F64[atoms] - fd) / scale
    emx = np.linalg.norm(Fmx[atoms] - fd) / scale
    ea = np.linalg.norm(Fmx[ace] - fd[: len(ace)]) / np.linalg.norm(fd[: len(ace)])
    print(f"FD on the full slab, {len(atoms)} atoms ({len(ace)} ACE, {len(pick)} EAM): fp64 {e64:.2e} "
          f"mixed {emx:.2e} (ACE atoms alone {ea:.2e})")
    assert e64 <= 1e-7
    assert emx <= 1e-5
    assert ea <= 1e-5
