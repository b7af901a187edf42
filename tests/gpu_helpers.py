"""Drive the HIP path through the C ABI for tests (marshalling only)."""
import numpy as np
import torch

from paper_2505_12958_amd import ap


def run_force(wl, precision=ap.AP_PREC_FP64, capacity=64, lam=None, with_eam=True, with_ace=True,
              virial=True, pos=None, with_rev=True, eam_analytic=None):
    """One AP force evaluation on the GPU: blend (unless lam given), neighbours,
    EAM, ACE.  Returns host numpy arrays."""
    dev = "cuda"
    N = wl.n_atoms
    S = ap.SystemsArg.from_workload(wl)
    p = wl.pos if pos is None else pos
    P = torch.tensor(np.ascontiguousarray(p.T), dtype=torch.float64, device=dev)
    ctx = ap.Context(wl.eam if with_eam and eam_analytic is None else None,
                     wl.ace if with_ace else None, precision)
    if with_eam and eam_analytic is not None:
        ctx.set_eam_analytic(eam_analytic)
    nl = ap.NeighbourList(N, capacity, dev, with_rev)
    ctx.build_neighbors(S, P, nl)
    lam_t = torch.zeros(N, dtype=torch.float64, device=dev)
    ace_list = torch.zeros(max(1, N), dtype=torch.int32, device=dev)
    n_ace = torch.zeros(1, dtype=torch.int32, device=dev)
    mask = (torch.tensor(wl.rule.mask, dtype=torch.uint8, device=dev)
            if wl.rule.mask is not None else None)
    if lam is None:
        ctx.blend(S, P, wl.rule, lam_t, ace_list, n_ace, mask)
    else:
        lam_t.copy_(torch.tensor(lam, dtype=torch.float64))
        idx = np.nonzero(np.asarray(lam) > 0)[0].astype(np.int32)
        ace_list[: len(idx)] = torch.tensor(idx, device=dev)
        n_ace.fill_(len(idx))
    e_atom = torch.zeros(N, dtype=torch.float64, device=dev)
    F = torch.zeros((3, N), dtype=torch.float64, device=dev)
    W = torch.zeros((wl.n_systems, 9), dtype=torch.float64, device=dev) if virial else None
    written = False
    if with_eam:
        ctx.eam_forces(S, P, nl, lam_t, e_atom, F, W)
        written = True
    if with_ace:
        ctx.ace_forces(S, P, nl, lam_t, ace_list, n_ace, e_atom, F, W, accumulate=written)
    e_sys = torch.zeros(wl.n_systems, dtype=torch.float64, device=dev)
    ctx.reduce_energy(S, e_atom, e_sys)
    torch.cuda.synchronize()
    ctx.check()
    na = int(n_ace.item())
    out = dict(e_atom=e_atom.cpu().numpy(), forces=F.cpu().numpy().T.copy(),
               e_sys=e_sys.cpu().numpy(), lam=lam_t.cpu().numpy(),
               ace_list=ace_list.cpu().numpy()[:na], nl=nl.rows(),
               count=nl.count.cpu().numpy()[:N])
    if with_rev:
        cnt = out["count"]
        rv = nl.rev.cpu().numpy().reshape(capacity, -1)[:, :N]
        out["rev"] = [rv[: cnt[i], i].copy() for i in range(N)]
    if virial:
        out["virial"] = W.cpu().numpy().reshape(-1, 3, 3)
    ctx.close()
    return out
