"""Velocity-Verlet steps of the FP64 path (ap_step: half kick, drift with
periodic wrap, indenter move, force evaluation with the switching rule
re-applied, half kick) against the oracle's vv_step driven by the oracle's
forces and indenter, on a small W slab with the tip pressed 1.5 A into the
surface; then the indenter energy and load of the final state against the
oracle's indenter (section "Nanoindentation": V_ind and the load equation).
Bar: 1e-10 relative on positions' displacements, velocities, energy and load."""
import numpy as np
import pytest
import torch

from oracle import md
from oracle.ap import APOracle, indenter
from oracle.geometry import Systems
from oracle.switching import lambda_of
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu

N_STEPS = 3


def test_vv_steps_and_indenter_match_oracle():
    wl = w.workload(3, scale=8)
    ind = dict(wl.indenter)
    ind["centre"] = np.asarray(ind["centre"], dtype=np.float64) - np.array([0.0, 0.0, 1.0])
    wl.indenter = ind
    mobile = wl.fixed == 0
    # tip in contact: atoms inside the sphere at the start
    d0 = np.linalg.norm(wl.pos - ind["centre"][None, :], axis=1)
    assert np.sum((d0 < ind["R"]) & mobile) >= 5

    ctx = ap.Context(wl.eam, wl.ace, ap.AP_PREC_FP64)
    st = ap.MD(wl)
    ctx.step(st.sys, st, 0)
    ctx.step(st.sys, st, N_STEPS)
    torch.cuda.synchronize()
    ctx.check()
    pos_g = st.pos.cpu().numpy().T
    vel_g = st.vel.cpu().numpy().T
    e_ind_g, load_g = float(st.e_ind.item()), float(st.load.item())
    centre_g = np.array(st.c.ind_centre[:])
    ctx.close()

    orc = APOracle(wl.eam, wl.ace)
    box = wl.box[0]

    def force_fn(x, c):
        S = Systems.from_workload(wl, pos=x)
        lam = lambda_of(x, wl.rule)
        out = orc.evaluate(S, lam, indenter_args=dict(ind, centre=c), mobile=mobile)
        return out["forces"]

    x, v, c = wl.pos.copy(), wl.vel.copy(), ind["centre"].copy()
    F = force_fn(x, c)
    for _ in range(N_STEPS):
        x, v, F, c = md.vv_step(x, v, F, wl.masses, wl.fixed, wl.dt, box, wl.periodic, force_fn,
                                ind_centre=c, ind_vel=ind["vel"])
    assert np.allclose(centre_g, c, rtol=0, atol=1e-12)
    # displacements (positions themselves are ~100 A) and velocities
    dx_ref = x - wl.pos
    dx_g = pos_g - wl.pos
    for k in range(3):
        if wl.periodic[k]:
            L = box[k][k]
            dx_ref[:, k] -= L * np.round(dx_ref[:, k] / L)
            dx_g[:, k] -= L * np.round(dx_g[:, k] / L)
    err_x = np.abs(dx_g - dx_ref).max() / np.abs(dx_ref).max()
    err_v = np.abs(vel_g - v).max() / np.abs(v).max()
    assert np.all(vel_g[wl.fixed != 0] == 0.0)
    E_ind, _, load = indenter(x, mobile, c, ind["R"], ind["K"])
    print(f"{N_STEPS} steps: displacement {err_x:.2e} velocity {err_v:.2e} "
          f"E_ind {e_ind_g:.6e} vs {E_ind:.6e}, load {load_g:.6e} vs {load:.6e}")
    assert err_x <= 1e-10 and err_v <= 1e-10
    assert E_ind > 0 and load > 0
    assert abs(e_ind_g - E_ind) <= 1e-10 * abs(E_ind)
    assert abs(load_g - load) <= 1e-10 * abs(load)
