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
