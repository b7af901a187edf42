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

Prints one JSON line.  value = atoms x steps / wall time of the timed steps,
timed with the library's phase timers off.  A second, separately timed pass
with the phase timers on gives the per-phase times and the duration of the
rank kernels (HIP events on the launch stream) for the roofline.  The
relative force error of the timed precision against the FP64 path is
measured on the same positions before timing; the FP64 path is timed too
(--fp64-steps 0 skips that timing).  A secondary number, `force_eval`, is the
median of 100 single force evaluations (no integration) timed with HIP events
after 10 warm-ups.

Roofline (algorithmic counts of the model, per phase):
  T_roof = sum over phases of max(bytes / 8 TB/s, VALU flops / 157.3 TFLOP/s
           (FP64: 78.6), MFMA flops / 2.5 PFLOP/s),
where the folded contraction is charged its three split products.  The
`roofline` object describes the dominant kernel family (the rank kernels):
its bound is the coupling and adjoint arithmetic on the vector ALUs; the
contraction's MFMA share is reported beside it.

Other workloads and the paper's AP-versus-ACE comparison:
--workload k selects one of the five synthetic workloads (5: the static
2.66M-atom slab); --mode ace / eam replaces the switching rule by lambda = 1
(pure ACE) / lambda = 0 (pure EAM) on the same atoms.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK = {"fp64_valu": 78.6, "fp32_valu": 157.3, "f16_mfma": 2500.0, "hbm": 8000.0}
SPLIT_PRODUCTS = 3


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    p.add_argument("--fp64-steps", type=int, default=5)
    p.add_argument("--force-evals", type=int, default=100,
                   help="single force evaluations timed for the secondary number (0 skips)")
    p.add_argument("--workload", type=int, default=3)
    p.add_argument("--mode", choices=["ap", "ace", "eam"], default="ap",
                   help="ap: the workload's switching rule; ace / eam: lambda = 1 / 0 everywhere")
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="CPU work of the oracle baseline sample, summed over cores (0 disables)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--pmc-probe", action="store_true",
                   help="for rocprofv3 --pmc runs: a 256 MiB elementwise kernel (counter "
                        "calibration), then three mixed force evaluations; prints nothing else")
    p.add_argument("--probe-key", default=None,
                   help="with --pmc-probe: write the workload key (name, mode, ACE atoms) here")
    p.add_argument("--record-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "KEY_JSON", "OUT"),
                   help="write the rank kernels' HBM traffic record from two --pmc runs of the probe")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(a, b):
    import torch
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def timed_steps(torch, ap, ctx, wl, steps, warmup, profile):
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


def force_evals(torch, ap, ctx, wl, n, warmup=10):
    """Median duration of n single force evaluations (ap_step with 0 steps),
    each bracketed by HIP events on the stream the library is called on."""
    if n <= 0:
        return None
    st = ap.MD(wl)
    for _ in range(warmup):
        ctx.step(st.sys, st, 0)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        ctx.step(st.sys, st, 0)
        b.record()
    torch.cuda.synchronize()
    ctx.check()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    med = ms[n // 2] if n % 2 else 0.5 * (ms[n // 2 - 1] + ms[n // 2])
    return {"evaluations": n, "median_ms": med, "min_ms": ms[0], "max_ms": ms[-1],
            "atom_evals_per_s": wl.n_atoms / (med * 1e-3)}


# ---------------------------------------------------------------- CPU baseline
def host_cores():
    """Cores this process may use, capped at 16 (the host CPU share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_chunk(args):
    """Worker: the oracle's neighbour search and bond terms for a chunk of
    atoms of the slab (one thread)."""
    k, atoms, kind = args
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.ap import APOracle
    from oracle.geometry import Systems
    from oracle.switching import lambda_of
    from paper_2505_12958_amd import workloads

    with threadpool_limits(limits=1):
        wl = _oracle_chunk.cache.get(k)
        if wl is None:
            wl = workloads.workload(k)
            S = Systems.from_workload(wl)
            _oracle_chunk.cache[k] = wl = (wl, S, S.neighbour_finder(), lambda_of(wl.pos, wl.rule),
                                           APOracle(wl.eam, wl.ace))
        w, S, find, lam, orc = wl
        t = time.perf_counter()
        nl = {int(i): find(int(i)) for i in atoms}
        if kind != "nbr":
            orc.bond_terms(S, lam, [int(i) for i in atoms], nl)
        return time.perf_counter() - t


_oracle_chunk.cache = {}


def start_pool(cores):
    """Worker processes for the oracle baseline, forked before anything in
    this process touches the GPU; each loads the workload once."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    return ctx.Pool(cores)


def cpu_baseline(pool, cores, wl, k, lam, budget_s):
    """The FP64 oracle on all `cores` host cores (one worker process each), on
    a bounded sample of the same slab: neighbour search of sampled atoms, bond
    terms of sampled EAM-only and ACE atoms.  The wall time of each sample
    class on all cores, scaled by the class's share of one full force
    evaluation, gives the oracle's atom-steps/s."""
    import numpy as np
    rng = np.random.default_rng(7)
    ace_atoms = np.nonzero(lam > 0)[0]
    eam_atoms = np.nonzero(lam == 0)[0]
    # warm the workers (workload generation is not timed)
    pool.map(_oracle_chunk, [(k, [0], "nbr")] * cores, chunksize=1)
    # per-atom cost estimates fix the sample sizes (about budget_s of CPU work)
    t_ace1 = pool.map(_oracle_chunk, [(k, [int(ace_atoms[0])], "ace")])[0]
    t_eam1 = max(1e-5, pool.map(_oracle_chunk, [(k, list(eam_atoms[:50]), "eam")])[0] / 50)
    n_ace_s = int(min(len(ace_atoms), max(cores, 0.7 * budget_s / max(t_ace1, 1e-4))))
    n_eam_s = int(min(len(eam_atoms), max(cores * 20, 0.2 * budget_s / t_eam1)))
    pa = rng.choice(ace_atoms, n_ace_s, replace=False)
    pe = rng.choice(eam_atoms, n_eam_s, replace=False)

    def wall(atoms, kind):
        chunks = [(k, list(c), kind) for c in np.array_split(atoms, cores) if len(c)]
        t = time.perf_counter()
        busy = sum(pool.map(_oracle_chunk, chunks, chunksize=1))
        return time.perf_counter() - t, busy

    t_a, busy_a = wall(pa, "ace")
    t_e, busy_e = wall(pe, "eam")
    N = wl.n_atoms
    # one full evaluation on all cores: each class scaled from its sample
    t_eval = t_a * len(ace_atoms) / n_ace_s + t_e * len(eam_atoms) / n_eam_s
    return {
        "value": N / t_eval, "unit": "atom-steps/s", "cores": cores, "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"FP64 numpy oracle in {cores} worker processes (one thread each, {cpu_model()}): "
                   f"neighbour search and bond terms of {n_ace_s} of the {len(ace_atoms)} ACE atoms "
                   f"({t_a:.1f} s wall, {busy_a:.0f} core-s) and of {n_eam_s} of the "
                   f"{len(eam_atoms)} EAM-only atoms ({t_e:.1f} s wall) of the same slab; each "
                   f"class scaled to its share of one full force evaluation "
                   f"({t_eval:.1f} s extrapolated)"),
    }


# ---------------------------------------------------------------- roofline
def roofline_model(ctx, ap, wl, n_ace, n_bonds, n_bonds_ace, fp64):
    """Algorithmic T_roof per phase (seconds) of one step, from the model's
    work counts.  Bytes are the compulsory HBM traffic of each phase: every
    input and output array once (neighbour positions inside a bond loop are
    gathers of arrays already counted)."""
    N = wl.n_atoms
    hbm = PEAK["hbm"] * 1e9
    valu = (PEAK["fp64_valu"] if fp64 else PEAK["fp32_valu"]) * 1e12
    f64 = PEAK["fp64_valu"] * 1e12
    mfma = PEAK["f16_mfma"] * 1e12
    ph = {}
    # neighbours: positions in (24 B), cell id/perm/cell copy (4+4+32 B),
    # list out (4 B per bond + count); canonical FP64 distance tests of ~20
    # flops against the 27 cells around each atom, whose occupancy follows
    # from the mean neighbour count (cells have edge r_c)
    rc = wl.cutoff
    occ = (n_bonds / max(1, N)) / (4.0 / 3.0 * 3.141592653589793 * rc ** 3) * rc ** 3
    ph["neighbors"] = max((N * (24 + 40 + 4) + 4 * n_bonds) / hbm, N * 27 * occ * 20 / f64)
    ph["blend"] = N * (24 + 8 + 4 + 1) / hbm
    # EAM: list read in both passes, positions, per-atom rho/F'/energy/force/virial
    ph["eam"] = max((2 * 4 * n_bonds + N * (24 + 8 * 4 + 24 + 72)) / hbm,
                    ctx.info("eam.flops_bond") * n_bonds / f64)
    ace_valu = ctx.info("ace.flops_atom") - ctx.info("ace.flops_contract")
    if fp64:
        ph["ace"] = (ctx.info("ace.flops_atom") * n_ace + ctx.info("ace.flops_bond") * n_bonds_ace) / valu
    else:
        ph["ace_bond"] = ctx.info("ace.flops_bond") * n_bonds_ace / valu
        # rank kernels: coupling and adjoint on the vector ALUs, then the
        # contraction's split products on MFMA (charged in sequence)
        ph["ace_rank_valu"] = ace_valu * n_ace / valu
        ph["ace_rank_mfma"] = SPLIT_PRODUCTS * ctx.info("ace.flops_contract") * n_ace / mfma
    # gather: per ACE bond the pair gradient (12 B) and 4 B of reverse-slot lookup (the atom-major
    # row copy the basis pass writes), per atom the force
    ph["ace_gather"] = (n_bonds_ace * 16 + N * 24) / hbm
    ph["indenter"] = N * (24 + 1 + 24) / hbm
    ph["integrate"] = 2 * N * (24 * 3 + 8 + 1) / hbm
    ph["reduce"] = N * 8 * 10 / hbm
    return ph


TRAFFIC_SOURCES = ["paper_2505_12958_amd/csrc/ace_rank.h", "paper_2505_12958_amd/csrc/k_ace_rank.hip",
                   "paper_2505_12958_amd/csrc/ap_internal.h", "paper_2505_12958_amd/csrc/ap_api.hip"]
COPY_BYTES = 256 * 1024 * 1024        # the probe's elementwise kernel reads and writes 256 MiB


def sources_sha256(paths):
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for src in paths:
        with open(os.path.join(here, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def record_traffic(fetch_csv, write_csv, key_json, out):
    """HBM bytes of one pass of the per-rank kernels from two rocprofv3 --pmc
    runs of `bench.py --pmc-probe` (FETCH_SIZE, then WRITE_SIZE, KB per
    dispatch), each scaled by what the counter reads for the probe's plain
    elementwise kernel of known size; written with the workload key and the
    kernel sources' hash."""
    import csv
    import re

    def per_kernel(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = re.sub(r"\(.*", "", r["Kernel_Name"])
            a = acc.setdefault(name, {})
            a[r["Dispatch_Id"]] = a.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        return {k: sum(v.values()) / len(v) for k, v in acc.items()}

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    # the calibration kernel: the torch elementwise kernel that moves the most bytes
    calib = sorted((k for k in fetch if "elementwise" in k.lower()), key=lambda k: -fetch[k])
    if not calib:
        raise SystemExit("no elementwise calibration kernel in the counter file")
    f_scale = COPY_BYTES / (fetch[calib[0]] * 1024.0)
    w_scale = COPY_BYTES / (write[calib[0]] * 1024.0)
    ranks = sorted(k for k in fetch if re.search(r"k_ace_rank<", k))
    fb = sum(fetch[k] for k in ranks) * 1024.0 * f_scale
    wb = sum(write.get(k, 0.0) for k in ranks) * 1024.0 * w_scale
    with open(key_json) as f:
        key = json.load(f)
    rec = {"kernel": "k_ace_rank<L>, one launch per coupled rank, one pass",
           "kernels": ranks, "key": key, "kernel_sources": TRAFFIC_SOURCES,
           "sources_sha256": sources_sha256(TRAFFIC_SOURCES),
           "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb,
           "calibration": {"fetch_scale": f_scale, "write_scale": w_scale, "kernel": calib[0],
                           "reference_bytes_each_way": COPY_BYTES,
                           "fetch_kb": fetch[calib[0]], "write_kb": write[calib[0]]}}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def recorded_traffic(prec, ap, key):
    """HBM bytes of one pass of the rank kernels from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (calibrated against a copy-type kernel),
    or None when the kernel sources or the workload differ from those the
    counters were taken on."""
    here = os.path.dirname(os.path.abspath(__file__))
    rec = os.path.join(here, "profiles", "ace_rank_traffic.json")
    if prec == ap.AP_PREC_FP64 or not os.path.exists(rec):
        return None
    with open(rec) as f:
        d = json.load(f)
    if "kernel_sources" not in d or "sources_sha256" not in d or d.get("key") != key:
        return None
    return d["traffic_bytes"] if sources_sha256(d["kernel_sources"]) == d["sources_sha256"] else None


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
    if args.record_traffic:
        record_traffic(*args.record_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    from paper_2505_12958_amd import workloads

    want_cpu = (not args.no_cpu_baseline and args.cpu_seconds > 0 and args.mode == "ap"
                and not args.pmc_probe)
    cores = host_cores()
    pool = start_pool(cores) if want_cpu else None   # before the GPU is touched

    import torch

    from paper_2505_12958_amd import ap

    if args.pmc_probe:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.mul(x, 2.0, out=y)  # reads 256 MiB, writes 256 MiB
        wl = workloads.workload(args.workload)
        if args.mode != "ap":
            wl.rule = workloads.LambdaRule(workloads.LAMBDA_CONST, value=1.0 if args.mode == "ace" else 0.0)
        ctx = ap.Context(wl.eam, wl.ace, ap.AP_PREC_MIXED)
        st = ap.MD(wl)
        for _ in range(3):
            ctx.step(st.sys, st, 0)
        torch.cuda.synchronize()
        if args.probe_key:
            with open(args.probe_key, "w") as f:
                json.dump({"workload": wl.name, "mode": args.mode, "n_ace": int(st.n_ace.item())}, f)
        return

    t_setup = time.perf_counter()
    wl = workloads.workload(args.workload)
    if args.mode != "ap":
        wl.rule = workloads.LambdaRule(workloads.LAMBDA_CONST, value=1.0 if args.mode == "ace" else 0.0)
    N = wl.n_atoms
    log(f"workload {wl.name}: {N} atoms, setup {time.perf_counter() - t_setup:.1f}s")

    prec = ap.AP_PREC_MIXED if args.precision == "mixed" else ap.AP_PREC_FP64
    fp64 = prec == ap.AP_PREC_FP64
    ctx64 = ap.Context(wl.eam, wl.ace, ap.AP_PREC_FP64)
    ctx = ctx64 if fp64 else ap.Context(wl.eam, wl.ace, prec)   # raises if unsupported

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
    n_bonds = int(ref.nl.count[:N].sum().item())
    n_bonds_ace = int(ref.nl.count[ace_idx].sum().item())
    lam = ref.lam.cpu().numpy()
    log(f"n_ace {n_ace}, bonds {n_bonds}, ACE bonds {n_bonds_ace}, force err {err_f:.3e}")
    del ref, test

    # headline: phase timers off
    _, dt, _ = timed_steps(torch, ap, ctx, wl, args.steps, args.warmup, profile=False)
    value = N * args.steps / dt
    # secondary: single force evaluations (blend, neighbours, EAM, ACE, indenter;
    # no integration), median over HIP-event-timed calls after warm-ups
    fe = force_evals(torch, ap, ctx, wl, args.force_evals)
    # phases and the rank kernels' duration: a separate pass with the timers on
    _, dt_prof, prof = timed_steps(torch, ap, ctx, wl, max(3, args.steps // 2), 1, profile=True)
    steps_prof = max(3, args.steps // 2)
    if not fp64 and args.fp64_steps > 0:
        _, dt64, _ = timed_steps(torch, ap, ctx64, wl, args.fp64_steps, 1, profile=False)
        v64 = N * args.fp64_steps / dt64
    else:
        v64 = value if fp64 else None

    phases = {k: round(v[0] / steps_prof, 4) for k, v in prof.items() if v[1]}
    ace_ms, ace_calls = prof["ace"]
    t_rank = ace_ms / max(1, ace_calls) * 1e-3            # one pass over all coupled ranks
    roof_ph = roofline_model(ctx, ap, wl, n_ace, n_bonds, n_bonds_ace, fp64)
    t_roof_step = sum(roof_ph.values())
    if fp64:
        flops = ctx.info("ace.flops_atom") * n_ace + ctx.info("ace.flops_bond") * n_bonds_ace
        achieved = flops / t_rank / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK["fp64_valu"], "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp64_valu"], "traffic": None, "kernel": "k_ace_fp64",
                "kernel_avg_ms": t_rank * 1e3, "flops_per_launch": flops}
    else:
        f_valu = (ctx.info("ace.flops_atom") - ctx.info("ace.flops_contract")) * n_ace
        f_mfma = ctx.info("ace.flops_contract") * n_ace
        a_valu = f_valu / t_rank / 1e12
        a_mfma = f_mfma / t_rank / 1e12
        t_roof_rank = roof_ph["ace_rank_valu"] + roof_ph["ace_rank_mfma"]
        key = {"workload": wl.name, "mode": args.mode, "n_ace": n_ace}
        roof = {
            "bound": "alu", "achieved": a_valu, "peak": PEAK["fp32_valu"], "unit": "TFLOP/s",
            "frac": a_valu / PEAK["fp32_valu"], "traffic": recorded_traffic(prec, ap, key),
            "kernel": "k_ace_rank<L>, L=0..8 (coupling and adjoint on the vector ALUs; "
                      "split-fp16 contraction on MFMA)",
            "kernel_avg_ms": t_rank * 1e3, "valu_flops_per_pass": f_valu,
            "mfma": {"achieved": a_mfma, "peak": PEAK["f16_mfma"], "unit": "TFLOP/s",
                     "frac": a_mfma / PEAK["f16_mfma"], "flops_per_pass": f_mfma,
                     "executed_flops_per_pass": ctx.info("ace.mfma_flops_atom") * n_ace},
            "t_roof_ms": t_roof_rank * 1e3, "t_roof_frac": t_roof_rank / t_rank,
            "launch_mode": ["one kernel per coupled rank", "all ranks in one persistent launch",
                            "all ranks in one persistent launch, device work counter"][
                int(ctx.info("ace.rank_mode"))],
        }
    roof["step"] = {"t_roof_ms": t_roof_step * 1e3, "ms_per_step": dt / args.steps * 1e3,
                    "frac": t_roof_step / (dt / args.steps),
                    "phases_t_roof_ms": {k: round(v * 1e3, 5) for k, v in roof_ph.items()}}

    line = {
        "metric": "AP force atom-steps/s at <=1e-5 rel force err vs FP64; % roofline; vs FP64 path",
        "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if fp64 else "mixed(f32 basis/coupling/adjoint, f16x3 split mfma, f64 sums/embedding/vv)",
        "data": "synthetic",
        "config": {"workload": describe(wl, args.mode, n_ace)},
        "force_rel_err_vs_fp64": err_f, "energy_rel_err_vs_fp64": err_e,
        "virial_rel_err_vs_fp64": err_w, "fp64_path_value": v64,
        "vs_fp64_path": value / v64 if v64 else None,
        "phase_ms_per_step": phases, "ms_per_step_profiled": dt_prof / steps_prof * 1e3,
        "force_eval": fe,
        "roofline": roof,
    }
    if pool is not None:
        log(f"timing the CPU oracle sample on {cores} cores ...")
        line["cpu_baseline"] = cpu_baseline(pool, cores, wl, args.workload, lam, args.cpu_seconds)
        pool.close()
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
