"""Seeded inputs: sizes of the workloads against the sizes the paper prints."""
import os

import numpy as np


def test_laplace_table_sizes_match_the_paper():
    """Every row of the paper's 125-ellipsoid table (Sec. 6.1) has N = 125 x
    N_G x N_F; the lattice workload built with N_G / 10 panels of 10 Gauss nodes
    and N_F = 2M + 1 azimuthal nodes has exactly that many unknowns, and its
    bodies fill [0, 10.2]^3 with neighbouring tips 0.05 apart."""
    from workloads import configs
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "laplace_125_spheroids_table.txt"))
    assert rows.shape == (8, 6)
    for N, NG, NF, *_ in rows:
        assert int(N) == 125 * int(NG) * int(NF)
        assert int(NF) % 2 == 1
        wl = configs.laplace_ellipsoids(n_panels=int(NG) // 10, p=10, M=(int(NF) - 1) // 2)
        assert wl.N == int(N)
    wl = configs.laplace_ellipsoids()
    lo = np.min([b.centre - np.array([0.5, 0.5, 1.0]) for b in wl.bodies], axis=0)
    hi = np.max([b.centre + np.array([0.5, 0.5, 1.0]) for b in wl.bodies], axis=0)
    assert np.all(lo >= 0.0) and np.all(hi <= 10.2 + 1e-12)
    assert np.isclose(lo[2], 0.0) and np.isclose(hi[2], 10.2)
    zs = sorted({b.centre[2] for b in wl.bodies})
    assert np.allclose(np.diff(zs) - 2.0, 0.05)
