"""The paper's W EAM in closed form on the GPU (ap_set_eam_analytic) against
the closed-form oracle: pure EAM on the periodic bulk and the AP energy with
ACE on the W slab (with the indenter's region and surface zone), forces,
per-atom energies and virial; FP64 <= 1e-10, mixed <= 1e-5."""
import numpy as np
import pytest

from gpu_helpers import run_force
from oracle.ap import APOracle
from oracle.eam_analytic import AnalyticWEam
from oracle.geometry import Systems
from oracle.switching import lambda_of
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu

PARAMS = dict(w.W_EAM, zbl=w.ZBL_C)


@pytest.mark.parametrize("name,k,scale,pure", [("bulk2000", 1, None, True), ("wslab10", 3, 10, False)])
@pytest.mark.parametrize("prec,tol", [(ap.AP_PREC_FP64, 1e-10), (ap.AP_PREC_MIXED, 1e-5)])
def test_closed_form_eam_matches_oracle(name, k, scale, pure, prec, tol):
    wl = w.workload(k) if scale is None else w.workload(k, scale=scale)
    lam = np.zeros(wl.n_atoms) if pure else lambda_of(wl.pos, wl.rule)
    S = Systems.from_workload(wl)
    ref = APOracle(None, None if pure else wl.ace, eam_model=AnalyticWEam(PARAMS)).evaluate(S, lam)
    g = run_force(wl, precision=prec, lam=lam, with_ace=not pure, eam_analytic=PARAMS)
    F, Fr = g["forces"], ref["forces"]
    if prec == ap.AP_PREC_FP64:
        ef = np.abs(F - Fr).max() / np.sqrt(np.mean(Fr ** 2))
    else:
        ef = np.linalg.norm(F - Fr) / np.linalg.norm(Fr)
    ee = np.abs(g["e_atom"] - ref["e_atom"]).max() / np.abs(ref["e_atom"]).max()
    ew = np.linalg.norm(g["virial"] - ref["virial"]) / np.linalg.norm(ref["virial"])
    print(f"{name} precision {prec}: force {ef:.2e} energy {ee:.2e} virial {ew:.2e}")
    assert ef <= tol and ee <= tol and ew <= tol
