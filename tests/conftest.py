import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def c1_system():
    """Oracle system of the two-sphere workload (kappa = pi, N = 8200)."""
    from oracle.multibody import System
    from workloads import configs
    wl = configs.two_spheres()
    return wl, System.from_workload(wl)


@pytest.fixture(scope="session")
def small_system():
    """A cheap two-body oracle system (sphere + rotated spheroid) for quick checks."""
    import numpy as np
    from oracle.multibody import System
    from workloads import configs, geometry as geo
    k = 2.0
    s = geo.sphere(1.0, 4, 10)
    pr = geo.prolate(0.8, 1.3, 5, 10)
    rot = geo.random_rotation(np.random.default_rng(7))
    wl = configs.Workload("small", k, k, [configs.BodySpec(s, np.array([0.0, 0.0, 0.0]), np.eye(3), 8),
                                        configs.BodySpec(pr, np.array([2.6, 0.4, -0.3]), rot, 8)],
                          np.array([[0.0, 0.6, 0.8]]))
    return wl, System.from_workload(wl)


@pytest.fixture(scope="session")
def laplace_system():
    """Zero frequency (kappa = 0, single-layer coefficient eta = 1, the Laplace equation
    of Sec. 6.1): sphere, rotated spheroid and rotated bowl."""
    import numpy as np
    from oracle.multibody import System
    from workloads import configs
    wl = configs.laplace_small()
    return wl, System.from_workload(wl)
