"""The W model (n_max 8, l_max 4, nu <= 4) at lambda = 1 on a 2,662-atom slab:
333 tiles of 8 ACE atoms over the one-per-compute-unit workgroups of the
rank kernels (256 on MI355X), so about 77 workgroups run a second tile at
every coupled rank L = 0..8 (the persistent loop's next-tile fetch and
staging).  Every atom's force, per-atom energy and the virial against the
oracle: FP64 <= 1e-10 (largest deviation over the RMS force), mixed <= 1e-5
(relative norm)."""
import numpy as np
import pytest
import torch

from gpu_helpers import run_force
from oracle.ap import APOracle
from oracle.geometry import Systems
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu

_REF = {}


def reference():
    if not _REF:
        wl = w.workload(3, scale=11)
        lam = np.ones(wl.n_atoms)
        S = Systems.from_workload(wl)
        _REF["wl"] = wl
        _REF["ref"] = APOracle(None, wl.ace).evaluate(S, lam)
    return _REF["wl"], _REF["ref"]


@pytest.mark.parametrize("prec", [ap.AP_PREC_FP64, ap.AP_PREC_MIXED])
def test_w_model_more_tiles_than_workgroups(prec):
    wl, ref = reference()
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    tiles = (wl.n_atoms + 7) // 8
    assert tiles > n_cu, (tiles, n_cu)
    g = run_force(wl, precision=prec, lam=np.ones(wl.n_atoms), with_eam=False)
    F, Fr = g["forces"], ref["forces"]
    rms = np.sqrt(np.mean(Fr ** 2))
    e_max = np.abs(F - Fr).max() / rms
    e_norm = np.linalg.norm(F - Fr) / np.linalg.norm(Fr)
    e_E = np.abs(g["e_atom"] - ref["e_atom"]).max() / np.abs(ref["e_atom"]).max()
    e_W = np.linalg.norm(g["virial"] - ref["virial"]) / np.linalg.norm(ref["virial"])
    print(f"precision {prec}: {tiles} tiles on {n_cu} CUs, force max {e_max:.2e} norm {e_norm:.2e}, "
          f"per-atom energy {e_E:.2e}, virial {e_W:.2e}")
    if prec == ap.AP_PREC_FP64:
        assert e_max <= 1e-10 and e_E <= 1e-10 and e_W <= 1e-10
    else:
        assert e_norm <= 1e-5 and e_E <= 1e-5 and e_W <= 1e-5
