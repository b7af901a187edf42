"""Mixed-precision HIP path (FP32 bond basis and coupling, split-fp16 MFMA
contraction with FP32 accumulation, FP64 displacements, embedding, sums)
against the FP64 oracle on the same positions.  Bar: relative RMS force
error <= 1e-5 (the path's accuracy target)."""
import numpy as np
import pytest

from gpu_helpers import run_force
from oracle.ap import APOracle
from oracle.geometry import Systems
from oracle.switching import lambda_of
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu

CASES = {"bulk2000": (1, None), "wslab10": (3, 10), "cuslab8": (2, 8), "batch6": (4, 6)}
_CACHE = {}


def case(name):
    if name not in _CACHE:
        k, sc = CASES[name]
        wl = w.workload(k) if sc is None else w.workload(k, scale=sc)
        S = Systems.from_workload(wl)
        lam = lambda_of(wl.pos, wl.rule)
        _CACHE[name] = (wl, APOracle(wl.eam, wl.ace).evaluate(S, lam))
    return _CACHE[name]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_forces_energy_virial(name):
    wl, ref = case(name)
    g = run_force(wl, precision=ap.AP_PREC_MIXED)
    ef = rel(g["forces"], ref["forces"])
    ee = float(np.abs(g["e_sys"] - ref["e_sys"]).max() / np.abs(ref["e_sys"]).max())
    ew = rel(g["virial"], ref["virial"])
    print(f"{name}: force {ef:.2e} energy {ee:.2e} virial {ew:.2e}")
    assert ef <= 1e-5
    assert ee <= 1e-5
    assert ew <= 1e-5


@pytest.mark.parametrize("name", ["bulk2000", "wslab10"])
def test_mixed_ace_component(name):
    """The ACE part alone (lambda = 1 everywhere, no EAM), so the error is not
    diluted by the EAM forces."""
    wl, _ = case(name)
    n = wl.n_atoms
    lam = np.ones(n)
    S = Systems.from_workload(wl)
    ref = APOracle(None, wl.ace).evaluate(S, lam)
    g = run_force(wl, precision=ap.AP_PREC_MIXED, lam=lam, with_eam=False)
    ef = rel(g["forces"], ref["forces"])
    ee = float(np.abs(g["e_atom"] - ref["e_atom"]).max() / np.abs(ref["e_atom"]).max())
    print(f"{name} ACE only: force {ef:.2e} per-atom energy {ee:.2e}")
    # the ACE part alone meets the path's accuracy target on its own
    assert ef <= 1e-5
    assert ee <= 1e-5


@pytest.mark.parametrize("precision,tol", [(ap.AP_PREC_FP64, 1e-10), (ap.AP_PREC_MIXED, 1e-5)])
@pytest.mark.parametrize("name", ["wslab10", "batch6"])
def test_md_force_evaluation(name, precision, tol):
    """The force evaluation of ap_step (EAM, then ACE adding its per-atom
    virial to the EAM call's before one reduction, on positions packed once)
    against the oracle, with the indenter off: forces, system energies and
    virials of a slab where both potentials contribute, and of a batch."""
    import torch
    wl, ref = case(name)
    ctx = ap.Context(wl.eam, wl.ace, precision)
    md = ap.MD(wl)
    md.c.ind_K = 0.0
    ctx.step(md.sys, md, 0)
    torch.cuda.synchronize()
    ctx.check()
    F = md.force.cpu().numpy().T
    W = md.virial.cpu().numpy().reshape(-1, 3, 3)
    E = md.e_sys.cpu().numpy()
    ctx.close()
    ef = rel(F, ref["forces"])
    ee = float(np.abs(E - ref["e_sys"]).max() / np.abs(ref["e_sys"]).max())
    ew = rel(W, ref["virial"])
    print(f"{name} precision {precision}: force {ef:.2e} energy {ee:.2e} virial {ew:.2e}")
    assert ef <= tol and ee <= tol and ew <= tol
