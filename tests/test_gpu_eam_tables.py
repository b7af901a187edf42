"""EAM with pair tables too large for the LDS stage of the EAM kernels (the
kernels then read them through the caches).  The tables are the generator's
piecewise cubics with every interval split in two (the same polynomial
re-expanded about the midpoint), so they define the same functions: forces and
energies must match the oracle on the original tables to the FP64 bar."""
import dataclasses

import numpy as np
import pytest

from gpu_helpers import run_force
from oracle.ap import APOracle
from oracle.geometry import Systems
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu

TOL = 1e-10


def split_intervals(t):
    """Each cubic a + b u + c u^2 + d u^3 on [0, dx] becomes two on [0, dx/2]:
    the first keeps its coefficients, the second is the same cubic about h = dx/2."""
    h = 0.5 * t.dx
    a, b, c, d = t.coef.T
    second = np.stack([a + h * (b + h * (c + h * d)), b + h * (2.0 * c + 3.0 * h * d), c + 3.0 * h * d, d], 1)
    coef = np.empty((2 * len(t.coef), 4))
    coef[0::2] = t.coef
    coef[1::2] = second
    return w.Table(x0=t.x0, dx=h, n_knots=2 * (t.n_knots - 1) + 1, coef=coef)


def test_eam_tables_beyond_lds_stage():
    wl = w.workload(3, scale=10)
    big = dataclasses.replace(wl.eam, phi=split_intervals(wl.eam.phi), rho=split_intervals(wl.eam.rho))
    # rho and phi together exceed the 40 KB the kernels stage in LDS
    assert 32 * (big.rho.n_knots - 1 + big.phi.n_knots - 1) > 40 * 1024
    wl_big = dataclasses.replace(wl, eam=big)
    lam = np.zeros(wl.n_atoms)  # pure EAM: every atom uses the tables
    ref = APOracle(wl.eam, None).evaluate(Systems.from_workload(wl), lam)
    g_small = run_force(wl, precision=ap.AP_PREC_FP64, with_ace=False, lam=lam)
    g_big = run_force(wl_big, precision=ap.AP_PREC_FP64, with_ace=False, lam=lam)
    rms = np.sqrt(np.mean(ref["forces"] ** 2))
    for name, g in (("LDS tables", g_small), ("cached tables", g_big)):
        df = np.abs(g["forces"] - ref["forces"]).max() / rms
        de = np.max(np.abs(g["e_sys"] - ref["e_sys"]) / np.abs(ref["e_sys"]))
        dw = np.abs(g["virial"] - ref["virial"]).max() / np.abs(ref["virial"]).max()
        print(f"{name}: force {df:.2e} energy {de:.2e} virial {dw:.2e}")
        assert df <= TOL and de <= TOL and dw <= TOL
