"""The nanoindentation driver on the GPU path (paper_2505_12958_amd.indentation;
section "Nanoindentation"): a small W slab of the paper's set-up under the
closed-form W EAM; the depth advances by v dt per step, the load recorded
after each chunk is the oracle's P_ind of the positions reached, and the
zero-pressure lattice constant leaves the crystal at a small pressure."""
import numpy as np
import pytest
import torch

from oracle.ap import indenter
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import indentation as ind
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu


def context():
    ctx = ap.Context(None, None, ap.AP_PREC_FP64)
    ctx.set_eam_analytic(dict(w.W_EAM, zbl=w.ZBL_C))
    return ctx


def test_indentation_run_records_depth_and_oracle_load():
    setup = dict(w.INDENT_W, h0=-0.5, speed=2.0e-3)      # reach contact within a few hundred steps
    wl = w.make_indentation(setup, n_cells=12, a=3.189)
    ctx = context()
    run = ind.IndentationRun(ctx, wl)
    run.equilibrate(300)
    rec = run.indent(1200, record_every=300)
    assert rec.shape == (4, 3)
    np.testing.assert_allclose(np.diff(rec[:, 1]), 300 * setup["speed"] * wl.dt, rtol=1e-9)
    torch.cuda.synchronize()
    x = run.md.pos.cpu().numpy().T
    c = np.array(run.md.c.ind_centre[:])
    _, _, load = indenter(x, wl.fixed == 0, c, wl.indenter["R"], wl.indenter["K"])
    print(f"depths {rec[:, 1]}, loads {rec[:, 2]}, oracle load {load:.6e}, layer T "
          f"{run.temperature(wl.nvt):.0f} K")
    assert rec[-1, 1] > 1.5 and load > 0.0
    assert abs(rec[-1, 2] - load) <= 1e-10 * load
    ctx.close()


def test_zero_pressure_lattice_constant_of_the_w_eam():
    ctx = context()
    a, hist = ind.lattice_constant_at(ctx, "bcc", w.W_EAM_A0, w.MASS_W, 300.0, 277.0 / ind.EV_A3_TO_GPA,
                                      n_cells=8, steps=2000)
    print("lattice constant iterations:", hist, "->", a)
    # a hot crystal at the 0 K lattice constant is under positive pressure
    assert hist[0][1] > 0.0
    assert abs(hist[-1][1]) < 0.3 * abs(hist[0][1])
    assert w.W_EAM_A0 < a < w.W_EAM_A0 * 1.005
    ctx.close()
