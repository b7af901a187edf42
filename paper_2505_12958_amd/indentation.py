"""Nanoindentation runs on the GPU path and the analysis of their load curves.

Section "Nanoindentation" (three groups: fixed bottom, Nose-Hoover layer,
NVE top; the spherical indenter V_ind moving at constant velocity; the load
P_ind, the total indenter force along the direction of motion) and the
Results subsections (the Hertzian load P_H = 4/3 E* R^(1/2) h^(3/2) fitted to
the elastic part of P_ind(h), the contact radius a_c = sqrt(h (2R - h)) and
the hardness p_m = P_ind / (pi a_c^2)).

Every MD step runs in the library (ap_step); this module drives it in
chunks, records (depth, load) and fits the curve on the host.  Depth h is
measured from the mean height of the top atomic plane at the start of the
indentation to the indenter's lowest point, positive below the surface.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import ap

EV_A3_TO_GPA = 160.21766208
ACC = 9.648533212e-3          # (eV/A/amu) -> A/fs^2
KB = 8.617333262e-5           # eV/K


def indentation_modulus(h, P, R, h_fit):
    """E* (eV/A^3) of the least-squares fit of P_H(h) to the loads with
    0 < h <= h_fit."""
    h = np.asarray(h, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    keep = (h > 0.0) & (h <= h_fit)
    if not keep.any():
        raise ValueError("no loads with 0 < h <= h_fit")
    col = (4.0 / 3.0) * math.sqrt(R) * np.power(h[keep], 1.5)
    sol, *_ = np.linalg.lstsq(col[:, None], P[keep], rcond=None)
    return float(sol[0])


def first_load_drop(h, P, drop=0.05, min_load=0.0, window=1):
    """Depth of the first point where the load, averaged over `window`
    consecutive records, falls below (1 - drop) times its running maximum
    after that maximum has passed min_load (the end of the elastic part), or
    None."""
    h = np.asarray(h, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    if window > 1:
        P = np.convolve(P, np.ones(window) / window, mode="same")
    peak = -np.inf
    for hk, Pk in zip(h, P):
        if Pk > peak:
            peak = Pk
        elif peak > min_load and Pk < (1.0 - drop) * peak:
            return float(hk)
    return None


def contact_radius(h, R):
    h = np.asarray(h, dtype=np.float64)
    return np.sqrt(np.maximum(h * (2.0 * R - h), 0.0))


def hardness(P, h, R):
    """Mean contact pressure (eV/A^3); NaN without contact."""
    area = math.pi * contact_radius(h, R) ** 2
    out = np.full(np.shape(area), np.nan)
    on = area > 0.0
    out[on] = np.asarray(P, dtype=np.float64)[on] / area[on]
    return out


def lattice_constant_at(ctx, lattice, a0, mass, T, bulk_modulus, n_cells=14, steps=4000,
                        iterations=2, tau=100.0):
    """Lattice constant of zero pressure at temperature T (a stand-in for the
    paper's NPT equilibration): NVT runs of a periodic crystal on the
    context's potential, the pressure p = (2K + tr W) / (3V) averaged over
    the second half of each run (W the virial, -dE/d strain), and the Newton
    step a <- a (1 + p / (3 B)) with the given bulk modulus (eV/A^3)."""
    from . import workloads as w
    a = float(a0)
    history = []
    for it in range(iterations):
        wl = w.make_crystal(lattice, n_cells, a, mass, 2.0 * T, seed=11 + it)
        md = ap.MD(wl)
        md.use_nvt(np.ones(wl.n_atoms, bool), T, tau)
        ctx.step(md.sys, md, 0)
        V = float(np.linalg.det(wl.box[0]))
        half, ps = steps // 2, []
        ctx.step(md.sys, md, half)
        for _ in range(half // 50):
            ctx.step(md.sys, md, 50)
            two_k = float((md.vel ** 2 * md.mass).sum().item()) / ACC
            tr_w = float(md.virial[0, 0].item() + md.virial[0, 4].item() + md.virial[0, 8].item())
            ps.append((two_k + tr_w) / (3.0 * V))
        ctx.check()
        p = float(np.mean(ps))
        history.append((a, p))
        a = a * (1.0 + p / (3.0 * bulk_modulus))
    return a, history


class IndentationRun:
    """The protocol on one slab workload (workloads.make_indentation): an
    equilibration with the indenter away and the thermostat on every mobile
    atom, then the indentation with the thermostat on the workload's layer.
    The context's potential (EAM tables or closed form, ACE, precision) is
    the caller's."""

    def __init__(self, ctx, wl, capacity=64, tau=None):
        setup = wl.meta["setup"]
        self.ctx, self.wl = ctx, wl
        self.T = float(setup["T"])
        self.tau = float(setup["tau"] if tau is None else tau)
        self.R = float(wl.indenter["R"])
        self.K = float(wl.indenter["K"])
        self.md = ap.MD(wl, capacity=capacity)
        self.md.c.check_every = 0
        self.top = None
        self.steps_done = 0
        self.records = []        # (step, depth, load)

    def equilibrate(self, n_steps, chunk=500, heat=math.sqrt(2.0)):
        """n_steps with the indenter away and every mobile atom thermostatted;
        velocities are first scaled by `heat` (a perfect lattice with Maxwell
        velocities at 2T relaxes to T by equipartition)."""
        md = self.md
        md.c.ind_K = 0.0
        vel = list(md.c.ind_vel)
        for k in range(3):
            md.c.ind_vel[k] = 0.0
        md.vel.mul_(heat)
        md.use_nvt(self.wl.fixed == 0, self.T, self.tau)
        self.ctx.step(md.sys, md, 0)
        done = 0
        while done < n_steps:
            k = min(chunk, n_steps - done)
            self.ctx.step(md.sys, md, k)
            self.ctx.check()
            done += k
        for k in range(3):
            md.c.ind_vel[k] = vel[k]

    def temperature(self, mask=None):
        """Kinetic temperature of the mobile atoms (or of `mask`)."""
        m = torch.tensor(self.wl.fixed == 0 if mask is None else mask, device=self.md.vel.device)
        two_k = float((self.md.vel[:, m] ** 2 * self.md.mass[m]).sum().item()) / ACC
        return two_k / (3.0 * int(m.sum().item()) * KB)

    def top_plane(self):
        """Mean height of the atoms of the initial top atomic plane."""
        z0 = self.wl.pos[:, 2]
        top = z0 > z0.max() - 0.25 * self.wl.meta["a"]
        return float(self.md.pos[2].cpu().numpy()[top].mean())

    def indent(self, n_steps, record_every=100):
        """Advance the indentation by n_steps (the first call switches the
        thermostat to the layer and the indenter on); appends
        (step, depth, load) every record_every steps."""
        md = self.md
        if self.top is None:
            self.top = self.top_plane()
            md.use_nvt(self.wl.nvt, self.T, self.tau)
            md.c.ind_K = self.K
            self.ctx.step(md.sys, md, 0)
        end = self.steps_done + n_steps
        while self.steps_done < end:
            k = min(record_every, end - self.steps_done)
            self.ctx.step(md.sys, md, k)
            self.steps_done += k
            torch.cuda.synchronize()
            self.ctx.check()
            depth = self.top - (md.c.ind_centre[2] - self.R)
            self.records.append((self.steps_done, depth, float(md.load.item())))
        return np.array(self.records)


def main(argv=None):
    """python -m paper_2505_12958_amd.indentation: the W set-up with the
    paper's closed-form W EAM (lambda = 0 everywhere), equilibration, then
    indentation to --depth; prints progress and a JSON summary with E* from
    the fit up to the first load drop."""
    import argparse
    import json
    import time

    from . import workloads as w

    ap_ = argparse.ArgumentParser()
    ap_.add_argument("--cells", type=int, default=w.INDENT_W["n_cells"])
    ap_.add_argument("--equil", type=int, default=20000)
    ap_.add_argument("--a", type=float, default=None,
                     help="lattice constant (default: the EAM's zero-pressure value at T)")
    ap_.add_argument("--depth", type=float, default=12.0)
    ap_.add_argument("--record", type=int, default=200)
    ap_.add_argument("--out", default=None)
    a = ap_.parse_args(argv)
    ctx = ap.Context(None, None, ap.AP_PREC_FP64)
    ctx.set_eam_analytic(dict(w.W_EAM, zbl=w.ZBL_C))
    lat = a.a
    if lat is None:
        # the paper's W EAM: a0 = 3.1837 A and B = 277 GPa (properties table)
        lat, hist = lattice_constant_at(ctx, "bcc", w.W_EAM_A0, w.MASS_W, w.INDENT_W["T"],
                                        277.0 / EV_A3_TO_GPA)
        print("zero-pressure lattice constant:", " -> ".join(f"{x:.5f} (p {p * EV_A3_TO_GPA:+.3f} GPa)"
                                                           for x, p in hist), f"-> {lat:.5f}", flush=True)
    wl = w.make_indentation(w.INDENT_W, n_cells=a.cells, a=lat)
    run = IndentationRun(ctx, wl, capacity=96)
    t0 = time.time()
    print(f"{wl.n_atoms} atoms, equilibrating {a.equil} steps", flush=True)
    run.equilibrate(a.equil)
    print(f"equilibrated in {time.time() - t0:.0f} s, mobile T {run.temperature():.0f} K", flush=True)
    setup = wl.meta["setup"]
    n = int(round((a.depth - setup["h0"]) / setup["speed"]))
    chunk = 10000
    t1 = time.time()
    while run.steps_done < n:
        rec = run.indent(min(chunk, n - run.steps_done), a.record)
        print(f"h {rec[-1, 1]:.2f} A  P {rec[-1, 2]:.2f} eV/A  T {run.temperature():.0f} K "
              f"({time.time() - t1:.0f} s)", flush=True)
    rec = np.array(run.records)
    h, P = rec[:, 1], rec[:, 2]
    # load drop of 10 % on the curve averaged over 0.5 A of depth
    win = max(1, int(round(0.5 / (setup["speed"] * a.record))))
    drop = first_load_drop(h, P, drop=0.10, min_load=50.0, window=win)
    h_fit = drop if drop is not None else float(h.max())
    E = indentation_modulus(h, P, run.R, h_fit)
    ms = (time.time() - t1) * 1e3 / n
    fits = {f"{hf:g}": indentation_modulus(h, P, run.R, hf) * EV_A3_TO_GPA
            for hf in (2.0, 4.0, 6.0, 8.0) if hf <= h.max() and np.any((h > 0) & (h <= hf))}
    pm = hardness(P, h, run.R) * EV_A3_TO_GPA
    late = h > (h_fit + 2.0)
    hard = (float(np.mean(pm[late])), float(np.std(pm[late]))) if late.any() else None
    out = dict(atoms=wl.n_atoms, lattice_constant=lat, steps=n, ms_per_step=ms, h_fit=h_fit, first_load_drop=drop,
               hardness_GPa_mean_std=hard,
               E_star_GPa=E * EV_A3_TO_GPA, E_star_GPa_by_h_fit=fits, top_plane=run.top,
               T_end=run.temperature(),
               curve=[[float(x) for x in r] for r in rec])
    print(json.dumps({k: v for k, v in out.items() if k != "curve"}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f)
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
