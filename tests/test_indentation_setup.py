"""Host side of the nanoindentation protocol: the slab builder against the
paper's set-up tables (atom counts, box edges, group heights, indenter
start), and the load-curve analysis of the package against the oracle's on
the same curves."""
import numpy as np
import pytest

from oracle import indentation as orc
from paper_2505_12958_amd import indentation as ind
from paper_2505_12958_amd import workloads as w


@pytest.mark.parametrize("setup,atoms,edge", [(w.INDENT_W, 1272112, 273.1), (w.INDENT_CU, 4000000, 364.2)])
def test_paper_set_up_sizes(setup, atoms, edge):
    n = setup["n_cells"]
    per_cell = 2 if setup["lattice"] == "bcc" else 4
    assert n ** 3 * per_cell == atoms                     # the tables' numbers of atoms
    # box edges: the tables' edges are those of the paper's relaxed lattices at
    # temperature, within 1 % of the workloads' lattice constants
    assert abs(n * setup["a"] - edge) < 0.01 * edge


@pytest.mark.parametrize("setup", [w.INDENT_W, w.INDENT_CU])
def test_groups_and_indenter_start(setup):
    wl = w.make_indentation(setup, n_cells=12)
    z = wl.pos[:, 2]
    z0 = z.min()
    fixed = wl.fixed != 0
    assert np.all(z[fixed] < z0 + setup["h_fixed"]) and np.all(z[~fixed] >= z0 + setup["h_fixed"])
    assert np.all(~wl.nvt[fixed])
    nv = wl.nvt
    assert np.all(z[nv] < z0 + setup["h_fixed"] + setup["h_nvt"])
    assert np.all(z[~fixed & ~nv] >= z0 + setup["h_fixed"] + setup["h_nvt"])
    assert np.all(wl.vel[fixed] == 0.0)
    c = wl.indenter["centre"]
    assert c[2] - setup["R"] - z.max() == pytest.approx(-setup["h0"], abs=1e-12)
    assert np.allclose(wl.indenter["vel"], [0.0, 0.0, -setup["speed"]])
    # the indenter starts clear of the surface
    assert np.linalg.norm(wl.pos - c[None, :], axis=1).min() > setup["R"]


def test_analysis_matches_oracle():
    R = 60.0
    rng = np.random.default_rng(9)
    h = np.linspace(-4.2, 14.0, 500)
    P = orc.hertz_load(h, 3.1, R)
    P = np.where(h > 8.3, 0.55 * P, P) + rng.normal(0.0, 2.0, h.shape)
    for h_fit in (3.0, 8.3):
        a = ind.indentation_modulus(h, P, R, h_fit)
        b = orc.hertz_fit(h, P, R, h_fit)
        assert abs(a - b) <= 1e-12 * abs(b)
    hd = ind.first_load_drop(h, orc.hertz_load(h, 3.1, R) * np.where(h > 8.3, 0.55, 1.0))
    assert hd is not None and 8.3 < hd < 8.3 + 2 * (h[1] - h[0])
    hp = np.array([-1.0, 0.5, 5.0, 12.0])
    Pp = np.array([0.0, 10.0, 200.0, 900.0])
    np.testing.assert_allclose(ind.contact_radius(hp, R), orc.contact_radius(hp, R), rtol=1e-15)
    np.testing.assert_allclose(ind.hardness(Pp, hp, R)[1:], orc.mean_contact_pressure(Pp, hp, R)[1:],
                               rtol=1e-14)
    assert np.isnan(ind.hardness(Pp, hp, R)[0])
    with pytest.raises(ValueError):
        ind.indentation_modulus(h, P, R, -5.0)
