"""The seeded input generators (shared by the library and the oracle, no
method arithmetic): determinism, ranges, and the grid form of the value
noise against its pointwise form."""
import numpy as np
import pytest

from paper_2403_15435_amd import inputs


@pytest.mark.parametrize("nx,ny,lx,ly,seed", [(129, 129, 2000.0, 2000.0, 2), (257, 129, 4000.0, 2000.0, 5),
                                              (65, 33, 640.0, 320.0, 4007)])
def test_value_noise_grid_equals_pointwise(nx, ny, lx, ly, seed):
    xs, ys = np.linspace(0.0, lx, nx), np.linspace(0.0, ly, ny)
    grid = inputs.value_noise(xs[None, :], ys[:, None], seed, base_wavelength=max(lx, ly) / 4.0)
    X, Y = np.broadcast_arrays(xs[None, :], ys[:, None])
    point = inputs.value_noise(X.copy(), Y.copy(), seed, base_wavelength=max(lx, ly) / 4.0)
    assert np.array_equal(grid, point)


def test_lattice_values_uniform_in_range():
    ix, iy = np.meshgrid(np.arange(-50, 50), np.arange(-50, 50))
    v = inputs.lattice_uniform(7, 3, ix, iy)
    assert v.min() >= -1.0 and v.max() < 1.0
    assert abs(v.mean()) < 0.05 and abs(v.var() - 1.0 / 3.0) < 0.02
    assert np.array_equal(v, inputs.lattice_uniform(7, 3, ix, iy))
    assert not np.array_equal(v, inputs.lattice_uniform(8, 3, ix, iy))


def test_fractal_dem_range_and_seed():
    a = inputs.fractal_dem_nodes(65, 65, 1000.0, 1000.0, seed=3)
    assert np.abs(a - 100.0).max() == pytest.approx(50.0, rel=1e-12)
    assert np.array_equal(a, inputs.fractal_dem_nodes(65, 65, 1000.0, 1000.0, seed=3))
    assert not np.array_equal(a, inputs.fractal_dem_nodes(65, 65, 1000.0, 1000.0, seed=4))
