"""Neighbour lists of a slab whose lower half is dense enough that the 27-cell
stencils there hold more candidates than the cell kernel stages in LDS (512),
so those atoms take the fallback kernel, while the sparse upper half stays on
the cell kernel.  Lists must equal the oracle's canonical rule bit for bit
(ascending j, strict r^2 < r_c^2, minimum image in x and y)."""
import numpy as np
import pytest
import torch

from oracle.geometry import Systems
from paper_2505_12958_amd import ap

pytestmark = pytest.mark.gpu

RC = 5.5
BOX = (30.0, 30.0, 40.0)
STAGE = 512  # candidates the cell kernel holds in LDS


def dense_over_sparse(seed=11):
    """Uniform random atoms: 0.11 per cubic angstrom for z < 20, 0.04 above."""
    rng = np.random.default_rng(seed)
    lx, ly, lz = BOX
    dense = rng.uniform((0.0, 0.0, 0.0), (lx, ly, 20.0), (int(lx * ly * 20.0 * 0.11), 3))
    sparse = rng.uniform((0.0, 0.0, 20.0), (lx, ly, lz), (int(lx * ly * 20.0 * 0.04), 3))
    pos = np.concatenate([dense, sparse])
    return pos[rng.permutation(len(pos))]


def stencil_totals(pos):
    """Candidates per cell (sum over its stencil), with the library's cell grid
    (edge >= r_c, periodic x and y, free z)."""
    g = [max(1, int(np.floor(L / (RC * (1.0 + 1e-9))))) for L in BOX]
    idx = np.minimum((pos / np.array(BOX) * g).astype(int), np.array(g) - 1)
    cnt = np.zeros(g, dtype=np.int64)
    np.add.at(cnt, tuple(idx.T), 1)
    tot = np.zeros_like(cnt)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                sh = np.roll(np.roll(cnt, -dx, 0), -dy, 1)
                if dz == 0:
                    tot += sh
                elif dz == 1:
                    tot[:, :, :-1] += sh[:, :, 1:]
                else:
                    tot[:, :, 1:] += sh[:, :, :-1]
    return tot


def test_dense_cells_fallback_bit_exact():
    pos = dense_over_sparse()
    n = len(pos)
    tot = stencil_totals(pos)
    # the case covers both kernels
    assert (tot > STAGE).any() and (tot <= STAGE).any()
    box = np.diag(BOX)
    ref = Systems(pos, box, [0, n], (True, True, False), RC).neighbour_lists_fast()
    cap = 128
    assert max(len(j) for j, _ in ref) <= cap
    S = ap.SystemsArg(box, [0, n], (True, True, False), RC)
    P = torch.tensor(np.ascontiguousarray(pos.T), dtype=torch.float64, device="cuda")
    ctx = ap.Context(None, None, ap.AP_PREC_FP64)
    try:
        for with_rev in (True, False):
            nl = ap.NeighbourList(n, cap, "cuda", with_rev)
            ctx.build_neighbors(S, P, nl)
            torch.cuda.synchronize()
            rows = nl.rows()
            bad = [i for i in range(n) if not np.array_equal(rows[i], ref[i][0])]
            print(f"dense/sparse slab: {n} atoms, {int((tot > STAGE).sum())} of {tot.size} cells "
                  f"over the LDS stage, rev={with_rev}, mismatched rows {len(bad)}")
            assert not bad, bad[:5]
            if with_rev:
                cnt = nl.count.cpu().numpy()[:n]
                rv = nl.rev.cpu().numpy().reshape(cap, -1)[:, :n]
                for i in range(0, n, 7):
                    for s, j in enumerate(rows[i]):
                        assert rows[j][rv[s, i]] == i
                assert np.array_equal(cnt, [len(j) for j, _ in ref])
    finally:
        ctx.close()
