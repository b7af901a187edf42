"""The nanoindentation protocol's Nose-Hoover layer on the GPU (ap_step with
st->nvt; section "Nanoindentation": fixed bottom, NVT layer above it, NVE
top, indenter moving into the surface) against the oracle's vv_step_nvt:
positions' displacements, velocities, the thermostat's xi and eta within
1e-10 relative, and the load P_ind of the final state."""
import numpy as np
import pytest
import torch

from oracle import md
from oracle.ap import APOracle, indenter
from oracle.eam_analytic import AnalyticWEam
from oracle.geometry import Systems
from oracle.switching import lambda_of
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu


def slab(hot):
    wl = w.workload(3, scale=10)                          # 2,000-atom W slab, fixed bottom 3 cells
    mobile = wl.fixed == 0
    z_fix = wl.pos[wl.fixed != 0, 2].max()
    layer = mobile & (wl.pos[:, 2] > z_fix) & (wl.pos[:, 2] <= z_fix + 10.0)
    if hot:
        wl.vel = wl.vel * np.sqrt(2.0)                    # 600 K against a 300 K thermostat
    return wl, layer


def compare(wl, pos_g, vel_g, x, v):
    dx_ref, dx_g = x - wl.pos, pos_g - wl.pos
    for k in range(2):
        L = wl.box[0][k][k]
        dx_ref[:, k] -= L * np.round(dx_ref[:, k] / L)
        dx_g[:, k] -= L * np.round(dx_g[:, k] / L)
    ex = np.abs(dx_g - dx_ref).max() / np.abs(dx_ref).max()
    ev = np.abs(vel_g - v).max() / np.abs(v).max()
    return ex, ev


def test_nvt_layer_with_closed_form_w_eam_matches_oracle():
    wl, layer = slab(hot=True)
    wl.ace = None
    wl.rule = w.LambdaRule(w.LAMBDA_CONST, value=0.0)     # EAM everywhere
    T0, tau, steps = 300.0, 10.0, 12
    ctx = ap.Context(None, None, ap.AP_PREC_FP64)
    ctx.set_eam_analytic(dict(w.W_EAM, zbl=w.ZBL_C))
    st = ap.MD(wl)
    st.c.ind_K = 0.0
    st.use_nvt(layer, T0, tau)
    ctx.step(st.sys, st, 0)
    ctx.step(st.sys, st, steps)
    torch.cuda.synchronize()
    ctx.check()
    pos_g, vel_g = st.pos.cpu().numpy().T, st.vel.cpu().numpy().T
    xi_g, eta_g = st.nvt_xi.cpu().numpy()[0]
    ctx.close()

    orc = APOracle(eam_model=AnalyticWEam(dict(w.W_EAM, zbl=w.ZBL_C)))
    lam = np.zeros(wl.n_atoms)

    def force_fn(x, c):
        return orc.evaluate(Systems.from_workload(wl, pos=x), lam)["forces"]

    x, v, xi, eta = wl.pos.copy(), wl.vel.copy(), 0.0, 0.0
    F = force_fn(x, None)
    for _ in range(steps):
        x, v, F, _, xi, eta = md.vv_step_nvt(x, v, F, wl.masses, wl.fixed, layer, xi, eta, wl.dt, T0,
                                             tau, wl.box[0], wl.periodic, force_fn)
    ex, ev = compare(wl, pos_g, vel_g, x, v)
    T_layer = md.layer_temperature(v, wl.masses, layer)
    print(f"{steps} NVT steps, {int(layer.sum())} layer atoms at {T_layer:.0f} K: displacement {ex:.1e} "
          f"velocity {ev:.1e} xi {xi_g:.6e} vs {xi:.6e} eta {eta_g:.6e} vs {eta:.6e}")
    assert xi > 0.0                                        # hot layer: the thermostat is pulling
    assert ex <= 1e-10 and ev <= 1e-10
    assert abs(xi_g - xi) <= 1e-10 * abs(xi) and abs(eta_g - eta) <= 1e-10 * abs(eta)
    assert np.all(vel_g[wl.fixed != 0] == 0.0)


def test_indentation_steps_with_nvt_layer_and_ap_match_oracle():
    """The whole protocol on the AP potential (tabulated EAM + ACE, FP64): NVE
    top under the moving indenter, NVT layer, fixed bottom."""
    wl, layer = slab(hot=False)
    ind = dict(wl.indenter)
    ind["centre"] = np.asarray(ind["centre"], dtype=np.float64) - np.array([0.0, 0.0, 1.0])
    wl.indenter = ind
    mobile = wl.fixed == 0
    T0, tau, steps = 300.0, 100.0, 3
    ctx = ap.Context(wl.eam, wl.ace, ap.AP_PREC_FP64)
    st = ap.MD(wl)
    st.use_nvt(layer, T0, tau)
    ctx.step(st.sys, st, 0)
    ctx.step(st.sys, st, steps)
    torch.cuda.synchronize()
    ctx.check()
    pos_g, vel_g = st.pos.cpu().numpy().T, st.vel.cpu().numpy().T
    xi_g, eta_g = st.nvt_xi.cpu().numpy()[0]
    load_g = float(st.load.item())
    ctx.close()

    orc = APOracle(wl.eam, wl.ace)

    def force_fn(x, c):
        out = orc.evaluate(Systems.from_workload(wl, pos=x), lambda_of(x, wl.rule),
                           indenter_args=dict(ind, centre=c), mobile=mobile)
        return out["forces"]

    x, v, c, xi, eta = wl.pos.copy(), wl.vel.copy(), ind["centre"].copy(), 0.0, 0.0
    F = force_fn(x, c)
    for _ in range(steps):
        x, v, F, c, xi, eta = md.vv_step_nvt(x, v, F, wl.masses, wl.fixed, layer, xi, eta, wl.dt, T0,
                                             tau, wl.box[0], wl.periodic, force_fn, ind_centre=c,
                                             ind_vel=ind["vel"])
    ex, ev = compare(wl, pos_g, vel_g, x, v)
    _, _, load = indenter(x, mobile, c, ind["R"], ind["K"])
    print(f"{steps} indentation steps: displacement {ex:.1e} velocity {ev:.1e} xi {xi_g:.3e} vs {xi:.3e} "
          f"load {load_g:.6e} vs {load:.6e}")
    assert ex <= 1e-10 and ev <= 1e-10
    assert abs(xi_g - xi) <= 1e-10 * abs(xi) and abs(eta_g - eta) <= 1e-10 * abs(eta)
    assert load > 0 and abs(load_g - load) <= 1e-10 * load
