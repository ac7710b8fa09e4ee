"""Host-side driver logic that needs no GPU."""
import numpy as np

from paper_2106_11143_amd.drivers import count_defects


def _zigzag(n, kinks_at=(), amp=1e-6, spacing=5e-6, seed=0):
    z = np.arange(n) * spacing
    s = np.array([(-1) ** k for k in range(n)], dtype=float)
    for k in kinks_at:  # flip the pattern after position k: one domain wall
        s[k + 1:] *= -1
    g = np.random.Generator(np.random.PCG64(seed))
    theta = 0.7
    x = amp * s * np.cos(theta) + 1e-9 * g.normal(size=n)
    y = amp * s * np.sin(theta) + 1e-9 * g.normal(size=n)
    perm = g.permutation(n)  # input order must not matter
    return x[perm], y[perm], z[perm]


def test_perfect_zigzag_has_no_defect():
    assert count_defects(*_zigzag(40)) == 0


def test_domain_walls_are_counted():
    assert count_defects(*_zigzag(40, kinks_at=(10,))) == 1
    assert count_defects(*_zigzag(60, kinks_at=(10, 30, 31))) == 3


def test_tiny_chains():
    assert count_defects([0.0, 1.0], [0.0, 0.0], [0.0, 1.0]) == 0
