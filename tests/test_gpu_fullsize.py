"""Full-size workloads in the configuration the benchmark times, checked on
sampled atoms the oracle computes one by one (brute-force neighbour lists of
each sampled atom and of its neighbours).  Neighbour lists bit-exact; FP64
forces <= 1e-10 relative; mixed forces <= 1e-5 relative (per sampled atom
set, against the norm of the sampled forces)."""
import numpy as np
import pytest
import torch

from oracle.ap import APOracle
from oracle.geometry import Systems
from oracle.switching import lambda_of
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu

_WL = {}


def wl_of(k):
    if k not in _WL:
        _WL[k] = w.workload(k)
    return _WL[k]


def gpu_eval(wl, precision):
    ctx = ap.Context(wl.eam, wl.ace, precision)
    st = ap.MD(wl)
    ctx.step(st.sys, st, 0)
    torch.cuda.synchronize()
    ctx.check()
    out = dict(forces=st.force.cpu().numpy().T.copy(), lam=st.lam.cpu().numpy(),
               e_atom=st.e_atom.cpu().numpy(), nl=st.nl, n_ace=int(st.n_ace.item()),
               ace_list=st.ace_list[: int(st.n_ace.item())].cpu().numpy())
    ctx.close()
    return out


def sample_atoms(wl, lam, n_ace, n_other, seed):
    rng = np.random.default_rng(seed)
    ace = np.nonzero(lam > 0)[0]
    other = np.nonzero(lam == 0)[0]
    pick = list(rng.choice(ace, size=min(n_ace, len(ace)), replace=False)) if len(ace) else []
    if len(other):
        pick += list(rng.choice(other, size=min(n_other, len(other)), replace=False))
    return sorted(int(i) for i in pick)


@pytest.mark.parametrize("k,n_ace,n_other", [(1, 6, 6), (2, 4, 8), (3, 64, 8), (4, 6, 0), (5, 3, 6)])
def test_fullsize_sampled_parity(k, n_ace, n_other):
    wl = wl_of(k)
    g64 = gpu_eval(wl, ap.AP_PREC_FP64)
    gmx = gpu_eval(wl, ap.AP_PREC_MIXED)
    S = Systems.from_workload(wl)
    lam = lambda_of(wl.pos, wl.rule)
    assert np.abs(g64["lam"] - lam).max() <= 1e-12
    assert np.array_equal(g64["ace_list"], np.nonzero(lam > 0)[0])
    atoms = sample_atoms(wl, lam, n_ace, n_other, 100 + k)
    # neighbour lists of the sampled atoms, bit-exact
    find = S.neighbour_finder()
    rows = {}
    cnt = g64["nl"].count.cpu().numpy()
    nb = g64["nl"].nbr.view(g64["nl"].capacity, -1)
    for i in atoms:
        rows[i] = nb[: cnt[i], i].cpu().numpy()
        js, _ = find(i)
        assert np.array_equal(rows[i], js), i
    orc = APOracle(wl.eam, wl.ace)
    F, e, _ = orc.forces_at(S, lam, atoms, find)
    if wl.indenter and wl.indenter.get("K", 0) > 0:
        from oracle.ap import indenter
        _, Fi, _ = indenter(wl.pos[atoms], wl.fixed[atoms] == 0, wl.indenter["centre"],
                            wl.indenter["R"], wl.indenter["K"])
        F = F + Fi
    scale = np.linalg.norm(F)
    err64 = np.linalg.norm(g64["forces"][atoms] - F) / scale
    errmx = np.linalg.norm(gmx["forces"][atoms] - F) / scale
    print(f"workload {k}: {len(atoms)} sampled atoms, fp64 {err64:.2e}, mixed {errmx:.2e}")
    assert err64 <= 1e-10
    assert errmx <= 1e-5
    assert np.abs(g64["e_atom"][atoms] - e).max() <= 1e-10 * max(1.0, np.abs(e).max())


def test_batch_smallest_cells_complete():
    """Triclinic batch (lambda = 1, pure ACE): energy, forces and virial of
    the three smallest cells against the full oracle evaluation of each cell
    on its own."""
    wl = wl_of(4)
    ctx = ap.Context(wl.eam, wl.ace, ap.AP_PREC_FP64)
    st = ap.MD(wl)
    ctx.step(st.sys, st, 0)
    torch.cuda.synchronize()
    F = st.force.cpu().numpy().T
    W = st.virial.cpu().numpy().reshape(-1, 3, 3)
    E = st.e_sys.cpu().numpy()
    ctx.close()
    sizes = np.diff(wl.sys_offset)
    for s in np.argsort(sizes, kind="stable")[:3]:
        lo, hi = int(wl.sys_offset[s]), int(wl.sys_offset[s + 1])
        S = Systems(wl.pos[lo:hi], wl.box[s:s + 1], [0, hi - lo], wl.periodic, wl.cutoff)
        ref = APOracle(wl.eam, wl.ace).evaluate(S, np.ones(hi - lo))
        eF = np.abs(F[lo:hi] - ref["forces"]).max() / np.sqrt(np.mean(ref["forces"] ** 2))
        eE = abs(E[s] - ref["e_sys"][0]) / abs(ref["e_sys"][0])
        eW = np.abs(W[s] - ref["virial"][0]).max() / np.abs(ref["virial"][0]).max()
        print(f"cell {s}: {hi - lo} atoms, F {eF:.1e} E {eE:.1e} W {eW:.1e}")
        assert eF <= 1e-10 and eE <= 1e-10 and eW <= 1e-10
