"""Launch modes of the mixed rank phase (one kernel per coupled rank; all
ranks in one persistent launch, tiles round-robin; the same with tiles from
a device work counter) against each other and against the oracle, for both
model shapes; and the tuner's cache file."""
import json
import os

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


def case(name):
    if name not in _REF:
        wl = w.workload(3, scale=10) if name == "wslab10" else w.workload(1)
        lam = np.ones(wl.n_atoms)
        ref = APOracle(None, wl.ace).evaluate(Systems.from_workload(wl), lam)
        _REF[name] = (wl, lam, ref)
    return _REF[name]


def forces_in_mode(wl, lam, mode, monkeypatch):
    monkeypatch.setenv("AP_RANK_MODE", str(mode))
    return run_force(wl, precision=ap.AP_PREC_MIXED, lam=lam, with_eam=False)


@pytest.mark.parametrize("name", ["wslab10", "bulk2000"])
def test_rank_modes_agree_and_match_oracle(name, monkeypatch):
    wl, lam, ref = case(name)
    out = {m: forces_in_mode(wl, lam, m, monkeypatch) for m in (0, 1, 2)}
    for m, g in out.items():
        e = np.linalg.norm(g["forces"] - ref["forces"]) / np.linalg.norm(ref["forces"])
        print(f"{name} mode {m}: force err vs oracle {e:.2e}")
        assert e <= 1e-5
    # the modes run the same arithmetic per rank; only the order in which the
    # wavefronts add their phi terms may differ
    for m in (1, 2):
        d = np.linalg.norm(out[m]["forces"] - out[0]["forces"]) / np.linalg.norm(out[0]["forces"])
        assert d <= 1e-6, (m, d)


def test_tuner_writes_and_reuses_its_cache(tmp_path, monkeypatch):
    wl, lam, _ = case("wslab10")
    cache = tmp_path / "tune.json"
    monkeypatch.delenv("AP_RANK_MODE", raising=False)
    monkeypatch.setenv("AP_AUTOTUNE_CACHE", str(cache))
    ctx = ap.Context(None, wl.ace, ap.AP_PREC_MIXED)
    S = ap.SystemsArg.from_workload(wl)
    P = torch.tensor(np.ascontiguousarray(wl.pos.T), dtype=torch.float64, device="cuda")
    nl = ap.NeighbourList(wl.n_atoms, 64)
    ctx.build_neighbors(S, P, nl)
    lam_t = torch.ones(wl.n_atoms, dtype=torch.float64, device="cuda")
    acl = torch.arange(wl.n_atoms, dtype=torch.int32, device="cuda")
    nac = torch.tensor([wl.n_atoms], dtype=torch.int32, device="cuda")
    e = torch.zeros(wl.n_atoms, dtype=torch.float64, device="cuda")
    F = torch.zeros((3, wl.n_atoms), dtype=torch.float64, device="cuda")
    ctx.ace_forces(S, P, nl, lam_t, acl, nac, e, F)
    torch.cuda.synchronize()
    mode = int(ctx.info("ace.rank_mode"))
    assert mode in (0, 1, 2)
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    (key, val), = entries.items()
    assert val == mode and "|ace 8 4 8 4 8 " in key and key.endswith(f"|b{wl.n_atoms.bit_length() - 1}")
    stamp = os.stat(cache).st_mtime_ns
    F1 = F.clone()
    ctx.close()
    # a new context reads the cache: same mode, no second tuning (file untouched)
    ctx2 = ap.Context(None, wl.ace, ap.AP_PREC_MIXED)
    ctx2.ace_forces(S, P, nl, lam_t, acl, nac, e, F)
    torch.cuda.synchronize()
    assert int(ctx2.info("ace.rank_mode")) == mode
    assert os.stat(cache).st_mtime_ns == stamp
    assert float(torch.linalg.norm(F - F1) / torch.linalg.norm(F1)) <= 1e-6
    ctx2.close()
