"""ap_blend_noalloc (the switching call that allocates nothing: static device
scratch) against ap_blend through the C ABI, on two calls in a row on one
context, the second with a smaller system: lambda bitwise equal, the ACE
lists and counts equal.  Also: a system above the static scratch's limit is
rejected before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu


def outputs(N):
    lam = torch.full((max(1, N),), -1.0, dtype=torch.float64, device="cuda")
    acl = torch.full((max(1, N),), -7, dtype=torch.int32, device="cuda")
    nac = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    return lam, acl, nac


def both(ctx, wl):
    N = wl.n_atoms
    S = ap.SystemsArg.from_workload(wl)
    P = torch.tensor(np.ascontiguousarray(wl.pos.T), dtype=torch.float64, device="cuda")
    mask = (torch.tensor(wl.rule.mask, dtype=torch.uint8, device="cuda")
            if wl.rule.mask is not None else None)
    ref, got = outputs(N), outputs(N)
    ctx.blend(S, P, wl.rule, *ref, mask)
    ctx.blend_noalloc(S, P, wl.rule, *got, mask)
    torch.cuda.synchronize()
    ctx.check()
    n_ref, n_got = int(ref[2].item()), int(got[2].item())
    return N, ref, got, n_ref, n_got


def test_noalloc_blend_matches_blend_twice_smaller_second():
    big = w.workload(3, scale=12)       # 3,456-atom W slab: hemisphere and CSP mask
    small = w.workload(1, scale=8)      # 1,024-atom periodic bulk: tapered sphere
    ctx = ap.Context(big.eam, None, ap.AP_PREC_FP64)
    for wl in (big, small):
        N, ref, got, n_ref, n_got = both(ctx, wl)
        print(f"{wl.name}: {N} atoms, {n_ref} with lambda > 0")
        assert 0 < n_ref < N
        assert n_got == n_ref
        assert torch.equal(got[0][:N], ref[0][:N])
        assert torch.equal(got[1][:n_ref], ref[1][:n_ref])
    ctx.close()


def test_noalloc_blend_rejects_systems_above_its_limit():
    wl = w.workload(1, scale=6)
    ctx = ap.Context(wl.eam, None, ap.AP_PREC_FP64)
    S = ap.SystemsArg.from_workload(wl)
    n_big = 4_000_001
    off = (C.c_int64 * 2)(0, n_big)
    S.c.n_atoms = n_big
    S.c.sys_offset = C.cast(off, C.POINTER(C.c_int64))
    P = torch.zeros((3, 1), dtype=torch.float64, device="cuda")
    lam, acl, nac = outputs(1)
    r = ap.rule_struct(wl.rule)
    st = ap.lib().ap_blend_noalloc(ctx.h, C.byref(S.c), ap._ptr(P), C.byref(r), ap._ptr(lam),
                                   ap._ptr(acl), ap._ptr(nac), ap._stream())
    assert st == ap.AP_ERR_ARG
    assert b"static scratch" in ap.lib().ap_last_error(ctx.h)
    torch.cuda.synchronize()
    assert int(nac.item()) == -7          # nothing was enqueued
    ctx.close()
