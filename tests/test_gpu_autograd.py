"""Differentiable energy through the C ABI: APEnergy (lambda frozen) gives
the oracle energy and, through autograd, minus the library's forces; the
given-lambda list (AP_LAMBDA_GIVEN) matches the rule's list."""
import numpy as np
import pytest
import torch

from oracle.ap import APOracle
from oracle.geometry import Systems
from oracle.switching import lambda_of
from paper_2505_12958_amd import ap
from paper_2505_12958_amd import workloads as w

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [(ap.AP_PREC_FP64, 1e-10), (ap.AP_PREC_MIXED, 1e-5)])
def test_ap_energy_autograd(precision, tol):
    wl = w.workload(3, scale=8)
    S = Systems.from_workload(wl)
    lam = lambda_of(wl.pos, wl.rule)
    ref = APOracle(wl.eam, wl.ace).evaluate(S, lam)
    ctx = ap.Context(wl.eam, wl.ace, precision)
    ev = ap.Evaluator(ctx, ap.SystemsArg.from_workload(wl))
    pos = torch.tensor(np.ascontiguousarray(wl.pos.T), dtype=torch.float64, device="cuda",
                       requires_grad=True)
    lam_t = torch.tensor(lam, dtype=torch.float64, device="cuda")
    E = ap.APEnergy.apply(pos, lam_t, ev)
    E.backward()
    grad = pos.grad.cpu().numpy().T
    Eref = float(ref["e_sys"].sum())
    assert abs(float(E) - Eref) <= tol * abs(Eref)
    F = ref["forces"]
    err = np.linalg.norm(-grad - F) / np.linalg.norm(F)
    print(f"precision {precision}: energy rel {abs(float(E) - Eref) / abs(Eref):.2e}, grad rel {err:.2e}")
    assert err <= tol
    ctx.close()


def test_given_lambda_list_matches_rule():
    wl = w.workload(1)
    ctx = ap.Context(wl.eam, wl.ace, ap.AP_PREC_FP64)
    S = ap.SystemsArg.from_workload(wl)
    N = wl.n_atoms
    pos = torch.tensor(np.ascontiguousarray(wl.pos.T), dtype=torch.float64, device="cuda")
    lam = torch.zeros(N, dtype=torch.float64, device="cuda")
    l1 = torch.zeros(N, dtype=torch.int32, device="cuda")
    n1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.blend(S, pos, wl.rule, lam, l1, n1)
    lam_before = lam.clone()
    l2 = torch.zeros(N, dtype=torch.int32, device="cuda")
    n2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = ap.lib().ap_blend(ctx.h, ap.C.byref(S.c), ap._ptr(pos), ap.C.byref(ap.given_rule()),
                           ap._ptr(lam), ap._ptr(l2), ap._ptr(n2), ap._stream())
    assert st == ap.AP_OK
    torch.cuda.synchronize()
    assert torch.equal(lam, lam_before)
    assert int(n1.item()) == int(n2.item()) > 0
    k = int(n1.item())
    assert torch.equal(l1[:k], l2[:k])
    ctx.close()
