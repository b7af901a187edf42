#!/usr/bin/env python
"""Benchmark of the AP force path on one MI355X.

One step = one velocity-Verlet step of ap_step on the 250,000-atom BCC W-like
indentation slab (50x50x50 cells, a = 3.165 A, x/y periodic, free top, three
fixed unit-cell layers, spherical indenter R = 40 A, K = 10 eV/A^3 moving
down, ACE n_max = 8, l_max = 4, nu <= 4, switching region = tip hemisphere of
radius 30 A + 5 A taper united with a centro-symmetry mask, about 8 % of the
atoms): switching parameter, cell-list neighbour rebuild, EAM, ACE with the
adjoint forces and virial, indenter, integration.  Inputs are seeded and
synthetic (paper_2505_12958_amd.workloads) and resident in HBM when the
timed region starts.

Prints one JSON line.  value = atoms x steps / wall time of the timed steps.
The relative force error of the timed precision against the FP64 path is
measured on the same positions before timing; the FP64 path is timed too
(--fp64-steps 0 skips that timing).

Other workloads and the paper's AP-versus-ACE comparison:
--workload k selects one of the five synthetic workloads (5: the static
2.66M-atom slab); --mode ace / eam replaces the switching rule by lambda = 1
(pure ACE) / lambda = 0 (pure EAM) on the same atoms.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

PEAK = {"fp64_valu": 78.6, "fp32_valu": 157.3, "bf16_mfma": 2500.0, "hbm": 8000.0}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    p.add_argument("--fp64-steps", type=int, default=5)
    p.add_argument("--workload", type=int, default=3)
    p.add_argument("--mode", choices=["ap", "ace", "eam"], default="ap",
                   help="ap: the workload's switching rule; ace / eam: lambda = 1 / 0 everywhere")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="budget of the oracle CPU-baseline sample (0 disables)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--pmc-probe", action="store_true",
                   help="for rocprofv3 --pmc runs: a 256 MiB elementwise kernel (counter "
                        "calibration), then three mixed force evaluations; prints nothing else")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def force_eval(ap, ctx, wl, st):
    ctx.step(st.sys, st, 0)


def rel_err(a, b):
    import torch
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def timed_steps(ap, torch, ctx, wl, steps, warmup, profile):
    st = ap.MD(wl)
    ctx.step(st.sys, st, 0)
    for _ in range(warmup):
        ctx.step(st.sys, st, 1)
    torch.cuda.synchronize()
    ctx.check()
    if profile:
        ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(st.sys, st, 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = None
    if profile:
        prof = ctx.profile_read()
        ctx.profile(False)
    ctx.check()
    return st, t1 - t0, prof


def cpu_baseline(wl, budget_s):
    """The FP64 oracle, single-threaded, on a bounded sample of the same slab:
    per-atom costs of neighbour search, EAM-only atoms and ACE atoms, scaled
    to one full force evaluation."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.ap import APOracle
    from oracle.geometry import Systems
    from oracle.switching import lambda_of

    with threadpool_limits(limits=1):
        S = Systems.from_workload(wl)
        lam = lambda_of(wl.pos, wl.rule)
        orc = APOracle(wl.eam, wl.ace)
        rng = np.random.default_rng(7)
        ace_atoms = np.nonzero(lam > 0)[0]
        eam_atoms = np.nonzero(lam == 0)[0]
        # neighbour lists of every sampled atom: k-d-tree candidates, canonical test
        from scipy.spatial import cKDTree
        n_ace_s = int(max(16, min(len(ace_atoms), 0.6 * budget_s / 0.02)))
        pick_a = rng.choice(ace_atoms, size=min(n_ace_s, len(ace_atoms)), replace=False)
        pick_e = rng.choice(eam_atoms, size=min(3000, len(eam_atoms)), replace=False)
        sub = np.concatenate([pick_a, pick_e])
        p = wl.pos.copy()
        size = np.array([wl.box[0][k][k] if wl.periodic[k] else 1e9 for k in range(3)])
        for k in range(3):
            if not wl.periodic[k]:
                p[:, k] -= p[:, k].min()
        t = time.perf_counter()
        tree = cKDTree(np.mod(p, size), boxsize=size)
        cand = tree.query_ball_point(np.mod(p[sub], size), wl.cutoff * (1 + 1e-6))
        nl = {}
        for ii, i in enumerate(sub):
            js = np.sort(np.asarray(cand[ii], dtype=np.int64))
            d = S.disp(int(i), js)
            r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            keep = (r2 < S.rc2) & (js != i)
            nl[int(i)] = (js[keep], d[keep])
        t_nbr = (time.perf_counter() - t) / len(sub)
        t = time.perf_counter()
        orc.bond_terms(S, lam, [int(i) for i in pick_e], nl)
        t_eam = (time.perf_counter() - t) / len(pick_e)
        t = time.perf_counter()
        orc.bond_terms(S, lam, [int(i) for i in pick_a], nl)
        t_ace = (time.perf_counter() - t) / len(pick_a)
    N = wl.n_atoms
    t_eval = N * t_nbr + len(eam_atoms) * t_eam + len(ace_atoms) * t_ace
    return {
        "value": N / t_eval, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 numpy oracle, 1 thread: k-d-tree neighbour lists of {len(sub)} sampled atoms, "
                   f"EAM terms of {len(pick_e)} EAM-only atoms, ACE terms of {len(pick_a)} of the "
                   f"{len(ace_atoms)} ACE atoms of the same 250k-atom slab; per-atom costs scaled "
                   f"to one force evaluation ({t_eval:.1f} s extrapolated)"),
    }


def recorded_traffic(prec, ap):
    """HBM bytes of one pass of the rank kernels from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (calibrated against a copy-type kernel), or
    None when the kernel source has changed since the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    rec = os.path.join(here, "profiles", "ace_rank_traffic.json")
    if prec == ap.AP_PREC_FP64 or not os.path.exists(rec):
        return None
    with open(rec) as f:
        d = json.load(f)
    # the kernels' traffic depends on their source and on the host-side plan
    # (tiles, strides, which ranks keep X_L), so every listed file is hashed
    if "kernel_sources" not in d or "sources_sha256" not in d:
        return None
    h = hashlib.sha256()
    for src in d["kernel_sources"]:
        with open(os.path.join(here, src), "rb") as f:
            h.update(f.read())
    return d["traffic_bytes"] if h.hexdigest() == d["sources_sha256"] else None


def describe(wl, mode, n_ace):
    m = wl.ace
    model = f"ACE n_max={m.n_max} l_max={m.l_max} nu<={m.nu_max}" if m is not None else "no ACE"
    lam = {"ap": "the switching rule", "ace": "lambda = 1 (pure ACE)", "eam": "lambda = 0 (pure EAM)"}[mode]
    kind = "indentation slab" if wl.n_systems == 1 and not all(wl.periodic) else (
        "periodic bulk" if wl.n_systems == 1 else f"batch of {wl.n_systems} triclinic cells")
    return (f"{wl.name}: {kind}, {wl.n_atoms} atoms, {model}, {lam}, {n_ace} ACE-active atoms, "
            f"neighbours rebuilt every step, velocity-Verlet dt={wl.dt:g} fs")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2505_12958_amd import ap, workloads

    if args.pmc_probe:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.mul(x, 2.0, out=y)  # reads 256 MiB, writes 256 MiB
        wl = workloads.workload(args.workload)
        ctx = ap.Context(wl.eam, wl.ace, ap.AP_PREC_MIXED)
        st = ap.MD(wl)
        for _ in range(3):
            ctx.step(st.sys, st, 0)
        torch.cuda.synchronize()
        return

    t_setup = time.perf_counter()
    wl = workloads.workload(args.workload)
    if args.mode != "ap":
        wl.rule = workloads.LambdaRule(workloads.LAMBDA_CONST, value=1.0 if args.mode == "ace" else 0.0)
    N = wl.n_atoms
    log(f"workload {wl.name}: {N} atoms, setup {time.perf_counter() - t_setup:.1f}s")

    prec = ap.AP_PREC_MIXED if args.precision == "mixed" else ap.AP_PREC_FP64
    ctx64 = ap.Context(wl.eam, wl.ace, ap.AP_PREC_FP64)
    try:
        ctx = ap.Context(wl.eam, wl.ace, prec) if prec != ap.AP_PREC_FP64 else ctx64
        probe = ap.MD(wl)
        ctx.step(probe.sys, probe, 0)
        torch.cuda.synchronize()
    except ap.APError as e:
        if e.status != ap.AP_ERR_UNSUPPORTED:
            raise
        log(f"mixed path unavailable ({e}); timing the FP64 path")
        prec, ctx = ap.AP_PREC_FP64, ctx64

    # accuracy of the timed precision against the FP64 path, same positions
    ref = ap.MD(wl)
    ctx64.step(ref.sys, ref, 0)
    test = ap.MD(wl)
    ctx.step(test.sys, test, 0)
    torch.cuda.synchronize()
    err_f = rel_err(test.force, ref.force)
    err_e = abs(float(test.e_sys.sum() - ref.e_sys.sum())) / abs(float(ref.e_sys.sum()))
    err_w = rel_err(test.virial, ref.virial)
    n_ace = int(ref.n_ace.item())
    ace_idx = ref.ace_list[:n_ace].long()
    n_bonds_ace = int(ref.nl.count[ace_idx].sum().item())
    log(f"n_ace {n_ace}, ACE bonds {n_bonds_ace}, force err {err_f:.3e}")

    st, dt, prof = timed_steps(ap, torch, ctx, wl, args.steps, args.warmup, profile=True)
    value = N * args.steps / dt
    if prec != ap.AP_PREC_FP64 and args.fp64_steps > 0:
        _, dt64, _ = timed_steps(ap, torch, ctx64, wl, args.fp64_steps, 1, profile=False)
        v64 = N * args.fp64_steps / dt64
    elif prec == ap.AP_PREC_FP64:
        v64 = value
    else:
        v64 = None

    # dominant kernel: the ACE contraction phase (FP64: k_ace_fp64, which also
    # does the bond basis; mixed: the nine k_ace_rank<L> launches, bracketed
    # together by one pair of HIP events on the launch stream)
    ace_ms, ace_calls = prof["ace"]
    avg_s = ace_ms / max(1, ace_calls) * 1e-3
    if prec == ap.AP_PREC_FP64:
        flops = ctx.info("ace.flops_atom") * n_ace + ctx.info("ace.flops_bond") * n_bonds_ace
        bound, peak, kernel = "alu", PEAK["fp64_valu"], "k_ace_fp64"
    else:
        flops = ctx.info("ace.flops_atom") * n_ace
        bound, peak, kernel = "mfma", PEAK["bf16_mfma"], "k_ace_rank<L>, L=0..8"
    achieved = flops / avg_s / 1e12 if avg_s > 0 else 0.0
    roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": recorded_traffic(prec, ap), "kernel": kernel,
            "kernel_avg_ms": avg_s * 1e3, "flops_per_launch": flops}
    if prec != ap.AP_PREC_FP64:
        ex = ctx.info("ace.mfma_flops_atom") * n_ace
        roof["mfma_executed_flops"] = ex
        roof["mfma_executed_frac"] = ex / avg_s / 1e12 / peak if avg_s > 0 else 0.0
    phases = {k: round(v[0] / max(1, v[1]), 4) for k, v in prof.items() if v[1]}

    line = {
        "metric": "AP force atom-steps/s at <=1e-5 rel force err vs FP64; % roofline; vs FP64 path",
        "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == ap.AP_PREC_FP64 else "mixed(f32+bf16x3 mfma, f64 sums/embedding/vv)",
        "data": "synthetic",
        "config": {"workload": describe(wl, args.mode, n_ace)},
        "force_rel_err_vs_fp64": err_f, "energy_rel_err_vs_fp64": err_e,
        "virial_rel_err_vs_fp64": err_w, "fp64_path_value": v64,
        "vs_fp64_path": value / v64 if v64 else None,
        "phase_ms_per_call": phases,
        "roofline": roof,
    }
    if not args.no_cpu_baseline and args.cpu_seconds > 0 and args.mode == "ap" and args.workload == 3:
        log("timing the CPU oracle sample ...")
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
