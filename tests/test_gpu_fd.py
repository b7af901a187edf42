"""Finite-difference checks through the C ABI: forces of the FP64 and mixed
paths against central differences (one Richardson step) of the FP64 GPU
energy, on 64 sampled atoms of a 2000-atom W slab (nu <= 4 ACE region,
indenter in contact).  Atoms whose |phi2| < 1e-4 sit on the kink of the
embedding guard and are not sampled."""
import numpy as np
import pytest
import torch

from oracle.ap import APOracle
from oracle.geometry import Systems
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu


def energy_fn(wl, lam):
    ctx = ap.Context(wl.eam, wl.ace, ap.AP_PREC_FP64)
    S = ap.SystemsArg.from_workload(wl)
    N = wl.n_atoms
    nl = ap.NeighbourList(N, 64)
    lam_t = torch.tensor(lam, dtype=torch.float64, device="cuda")
    idx = np.nonzero(lam > 0)[0].astype(np.int32)
    acl = torch.zeros(N, dtype=torch.int32, device="cuda")
    acl[: len(idx)] = torch.tensor(idx, device="cuda")
    nac = torch.tensor([len(idx)], dtype=torch.int32, device="cuda")
    e_atom = torch.zeros(N, dtype=torch.float64, device="cuda")
    F = torch.zeros((3, N), dtype=torch.float64, device="cuda")
    e_sys = torch.zeros(1, dtype=torch.float64, device="cuda")
    e_ind = torch.zeros(1, dtype=torch.float64, device="cuda")
    fixed = torch.tensor(wl.fixed, dtype=torch.uint8, device="cuda")
    ind = wl.indenter

    def E(pos):
        P = torch.tensor(np.ascontiguousarray(pos.T), dtype=torch.float64, device="cuda")
        ctx.build_neighbors(S, P, nl)
        ctx.eam_forces(S, P, nl, lam_t, e_atom, F)
        ctx.ace_forces(S, P, nl, lam_t, acl, nac, e_atom, F, accumulate=True)
        ctx.reduce_energy(S, e_atom, e_sys)
        ctx.indenter(S, P, fixed, ind["centre"], ind["R"], ind["K"], F, e_ind=e_ind)
        return float(e_sys.item() + e_ind.item())
    return E


def forces(wl, precision):
    ctx = ap.Context(wl.eam, wl.ace, precision)
    st = ap.MD(wl)
    ctx.step(st.sys, st, 0)
    torch.cuda.synchronize()
    return st.force.cpu().numpy().T.copy(), st.lam.cpu().numpy()


def test_forces_match_fd_of_fp64_energy():
    wl = w.workload(3, scale=10)
    F64, lam = forces(wl, ap.AP_PREC_FP64)
    Fmx, _ = forces(wl, ap.AP_PREC_MIXED)
    E = energy_fn(wl, lam)
    rng = np.random.default_rng(3)
    ace = rng.permutation(np.nonzero(lam > 0)[0])
    S = Systems.from_workload(wl)
    nl = {int(i): S.neighbours_of(int(i)) for i in ace[:80]}
    _, _, _, _, phi = APOracle(None, wl.ace).bond_terms(S, lam, [int(i) for i in ace[:80]], nl)
    ace = [int(i) for i, ph in zip(ace[:80], phi) if abs(ph[1]) >= 1e-4][:48]
    atoms = ace + list(rng.choice(np.nonzero(lam == 0)[0], 64 - len(ace), replace=False))
    h = 2e-4
    fd = np.zeros((len(atoms), 3))
    for t, i in enumerate(atoms):
        for k in range(3):
            def d(hh):
                p = wl.pos.copy(); p[i, k] += hh
                m = wl.pos.copy(); m[i, k] -= hh
                return (E(p) - E(m)) / (2 * hh)
            fd[t, k] = -(4 * d(h / 2) - d(h)) / 3
    scale = np.linalg.norm(fd)
    e64 = np.linalg.norm(F64[atoms] - fd) / scale
    emx = np.linalg.norm(Fmx[atoms] - fd) / scale
    print(f"FD: fp64 {e64:.2e} mixed {emx:.2e}")
    assert e64 <= 1e-7
    assert emx <= 1e-5
