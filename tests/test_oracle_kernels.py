"""Pins for the oracle's Green's-function kernels (Section 4.2) against
central differences of G and against symmetry."""
import numpy as np
import pytest

from oracle import oracle as O


def _G(k, x, y):
    r = np.linalg.norm(np.asarray(x) - np.asarray(y))
    return np.exp(1j * k * r) / (4 * np.pi * r)


@pytest.mark.parametrize("k", [0.0, 3.0, 40.0])
def test_kernels_match_finite_differences(k):
    rng = np.random.default_rng(int(k) + 1)
    h = 1e-5
    for _ in range(20):
        x = rng.normal(size=3)
        y = x + rng.normal(size=3) * 0.3
        nx = rng.normal(size=3)
        nx /= np.linalg.norm(nx)
        ny = rng.normal(size=3)
        ny /= np.linalg.norm(ny)
        G, dny, dnx, dd = O.kernels(k, x, nx, y, ny)
        assert G == pytest.approx(_G(k, x, y), rel=1e-14)
        fd_ny = (_G(k, x, y + h * ny) - _G(k, x, y - h * ny)) / (2 * h)
        fd_nx = (_G(k, x + h * nx, y) - _G(k, x - h * nx, y)) / (2 * h)
        assert abs(dny - fd_ny) <= 1e-6 * abs(fd_ny) + 1e-9
        assert abs(dnx - fd_nx) <= 1e-6 * abs(fd_nx) + 1e-9

        def dGdny_at(xx):
            return O.kernels(k, xx, nx, y, ny)[1]
        fd_dd = (dGdny_at(x + h * nx) - dGdny_at(x - h * nx)) / (2 * h)
        assert abs(dd - fd_dd) <= 1e-5 * abs(fd_dd) + 1e-8


def test_kernel_symmetries():
    rng = np.random.default_rng(3)
    for _ in range(10):
        x, y = rng.normal(size=3), rng.normal(size=3)
        nx, ny = rng.normal(size=3), rng.normal(size=3)
        a = O.kernels(5.0, x, nx, y, ny)
        b = O.kernels(5.0, y, ny, x, nx)
        assert a[0] == b[0]                           # G symmetric
        assert a[1] == pytest.approx(b[2], rel=1e-13)  # dG/dn_y(x,y) = dG/dn_x(y,x)
        assert a[3] == pytest.approx(b[3], rel=1e-12)  # hypersingular kernel symmetric


def test_kernel_time_convention_outgoing():
    # G = e^{ikr}/(4 pi r): phase increases with r (outgoing for e^{-i w t})
    x = np.zeros(3)
    g1 = O.kernels(2.0, x, [0, 0, 1.0], [0.1, 0, 0], [1.0, 0, 0])[0]
    g2 = O.kernels(2.0, x, [0, 0, 1.0], [0.2, 0, 0], [1.0, 0, 0])[0]
    assert np.angle(g2) - np.angle(g1) == pytest.approx(0.2, rel=1e-12)
