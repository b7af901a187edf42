"""Dynamic switching (ap_switching_update; section "Adaptive-precision
potential" and the appendix "Switching function") against the oracle's
DynamicSwitching over several updates with moving positions: the averaged
CSP bit for bit, lambda within 1e-12 and the ACE lists identical; and
velocity-Verlet steps of ap_step with the dynamic rule against the oracle's
steps with the oracle's rule."""
import numpy as np
import pytest
import torch

from oracle import md
from oracle.ap import APOracle
from oracle.geometry import Systems
from oracle.switching import DynamicSwitching as OracleSwitching
from oracle.switching import SwitchParams, csp_all
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu


def setup(seed=0):
    wl = w.workload(3, scale=10)                          # 2,000-atom W slab, 31.65 A wide
    S = Systems.from_workload(wl)
    rows = S.neighbour_lists()
    c = csp_all(S, rows)
    bulk = np.array([len(r[0]) >= 50 for r in rows])
    z_top = wl.pos[:, 2].max()
    # thresholds in the tail of the bulk atoms' thermal CSP so the ramp and the
    # transition zone are exercised on a small slab (the free bottom surface
    # is detected as well)
    p = SwitchParams(csp_lo=float(np.quantile(c[bulk], 0.97)), csp_hi=float(np.quantile(c[bulk], 0.995)),
                     n_csp_avg=3, n_lambda_avg=2, r_lo=2.0, r_hi=6.0, dlambda_min=0.01,
                     centre=tuple(wl.indenter["centre"][:2]) + (z_top,), r_precise=6.0,
                     z_surface_min=z_top - 2.0)
    return wl, p


def gpu_switching(wl, p):
    return ap.DynamicSwitching(wl.n_atoms, csp_lo=p.csp_lo, csp_hi=p.csp_hi, n_csp=p.n_csp,
                               n_csp_avg=p.n_csp_avg, r_lo=p.r_lo, r_hi=p.r_hi,
                               n_lambda_avg=p.n_lambda_avg, dlambda_min=p.dlambda_min,
                               centre=p.centre, r_precise=p.r_precise, z_surface_min=p.z_surface_min)


def moved(wl, k):
    x = wl.pos + np.random.default_rng(50 + k).normal(0, 0.02, wl.pos.shape)
    for d in range(2):
        L = wl.box[0][d][d]
        x[:, d] = np.mod(x[:, d], L)
    return x


def test_switching_updates_match_oracle():
    wl, p = setup()
    N = wl.n_atoms
    ctx = ap.Context(wl.eam, None, ap.AP_PREC_FP64)
    S_arg = ap.SystemsArg.from_workload(wl)
    nl = ap.NeighbourList(N, 64, with_rev=False)
    sw = gpu_switching(wl, p)
    lam = torch.zeros(N, dtype=torch.float64, device="cuda")
    acl = torch.zeros(N, dtype=torch.int32, device="cuda")
    nac = torch.zeros(1, dtype=torch.int32, device="cuda")
    orc = OracleSwitching(p)
    for k in range(4):
        x = moved(wl, k)
        P = torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float64, device="cuda")
        ctx.build_neighbors(S_arg, P, nl)
        ctx.switching_update(S_arg, P, nl, sw, lam, acl, nac)
        torch.cuda.synchronize()
        ctx.check()
        lam_ref = orc.update(Systems.from_workload(wl, pos=x))
        c_gpu = sw.csp_avg.cpu().numpy()[:N]
        l_gpu = lam.cpu().numpy()
        n = int(nac.item())
        frac = np.mean(lam_ref > 0)
        print(f"update {k}: lambda > 0 on {n} atoms ({frac:.2%}), 0 < lambda < 1 on "
              f"{int(np.sum((lam_ref > 0) & (lam_ref < 1)))}, max |dlambda| {np.abs(l_gpu - lam_ref).max():.1e}")
        assert np.array_equal(c_gpu, orc.c_avg)                    # bit for bit
        assert np.abs(l_gpu - lam_ref).max() <= 1e-12
        assert np.array_equal(acl.cpu().numpy()[:n], np.nonzero(lam_ref > 0)[0])
        assert 0.02 < frac < 0.98
        assert np.sum((lam_ref > 0) & (lam_ref < 1)) > 10
    assert sw.c.initialised == 1
    ctx.close()


def test_md_steps_with_dynamic_switching_match_oracle():
    wl, p = setup()
    mobile = wl.fixed == 0
    ctx = ap.Context(wl.eam, wl.ace, ap.AP_PREC_FP64)
    st = ap.MD(wl)
    sw = gpu_switching(wl, p)
    st.use_switching(sw)
    ctx.step(st.sys, st, 0)
    ctx.step(st.sys, st, 3)
    torch.cuda.synchronize()
    ctx.check()
    pos_g, vel_g = st.pos.cpu().numpy().T, st.vel.cpu().numpy().T
    lam_g = st.lam.cpu().numpy()
    ctx.close()

    orc_sw = OracleSwitching(p)
    orc = APOracle(wl.eam, wl.ace)
    ind = wl.indenter
    last = {}

    def force_fn(x, c):
        S = Systems.from_workload(wl, pos=x)
        lam = orc_sw.update(S)
        last["lam"] = lam
        return orc.evaluate(S, lam, indenter_args=dict(ind, centre=c), mobile=mobile)["forces"]

    x, v, c = wl.pos.copy(), wl.vel.copy(), np.asarray(ind["centre"], dtype=np.float64)
    F = force_fn(x, c)
    for _ in range(3):
        x, v, F, c = md.vv_step(x, v, F, wl.masses, wl.fixed, wl.dt, wl.box[0], wl.periodic, force_fn,
                                ind_centre=c, ind_vel=ind["vel"])
    dx_ref, dx_g = x - wl.pos, pos_g - wl.pos
    for k in range(2):
        L = wl.box[0][k][k]
        dx_ref[:, k] -= L * np.round(dx_ref[:, k] / L)
        dx_g[:, k] -= L * np.round(dx_g[:, k] / L)
    ex = np.abs(dx_g - dx_ref).max() / np.abs(dx_ref).max()
    ev = np.abs(vel_g - v).max() / np.abs(v).max()
    print(f"3 steps with dynamic switching: displacement {ex:.1e} velocity {ev:.1e}, "
          f"lambda {np.abs(lam_g - last['lam']).max():.1e}, ACE atoms {int(np.sum(lam_g > 0))}")
    assert np.abs(lam_g - last["lam"]).max() <= 1e-12
    assert ex <= 1e-10 and ev <= 1e-10
