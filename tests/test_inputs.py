"""Seeded synthetic workloads: determinism, shapes and coverage targets."""
import numpy as np
import pytest

from paper_2404_12968_amd import inputs as I


def test_parity64_shape_and_determinism():
    a, b = I.parity64(), I.parity64()
    assert (a.nx, a.ny, a.alpha, a.kappa, a.sigma) == (64, 64, 1, 0.2, 0.1)
    assert a.cells.size == 205 and np.unique(a.cells).size == 205
    assert np.array_equal(a.cells, b.cells) and np.array_equal(a.y, b.y)
    assert a.bc_x == a.bc_y == I.BC_NEUMANN and a.dtype == "f64"


@pytest.mark.parametrize("fn,target", [(I.tracks2048, 0.08), (I.warm1024, 0.06)])
def test_track_coverage_within_one_percent(fn, target):
    p = fn()
    assert abs(p.coverage - target) <= 0.01
    assert p.cells.min() >= 0 and p.cells.max() < p.n
    assert np.all(np.diff(p.cells) > 0)


def test_global_grid_coverage_and_boundary():
    p = I.global8192()
    assert (p.nx, p.ny) == (8192, 4096)
    assert p.bc_x == I.BC_PERIODIC and p.bc_y == I.BC_NEUMANN
    assert abs(p.coverage - 0.05) <= 0.01


def test_tracks_wrap_in_x():
    rng = np.random.default_rng(0)
    cells = I.track_cells(10, 30, 1, 3, rng)
    xs, ys = cells % 10, cells // 10
    assert set(np.unique(ys)) == set(range(30))
    assert np.all(np.bincount(ys) == 3)


def test_batch_draws_follow_ranges():
    b = I.batch256(count=12)
    for p in b:
        assert 64 <= p.nx <= 1024 and p.nx == p.ny
        assert p.alpha in (1, 2) and 0.02 <= p.kappa <= 0.3 and 0.02 <= p.sigma <= 0.2
        assert 0.0095 <= p.coverage <= 0.2005
    again = I.batch256(count=12)
    assert all(np.array_equal(x.y, z.y) for x, z in zip(b, again))


def test_spectral_field_unit_variance_and_seeded():
    f1 = I.spectral_field(64, 48, 0.1, 2, np.random.default_rng(3))
    f2 = I.spectral_field(64, 48, 0.1, 2, np.random.default_rng(3))
    assert f1.shape == (48, 64) and np.array_equal(f1, f2)
    assert abs(f1.std() - 1.0) < 1e-12 and abs(f1.mean()) < 1e-12


def test_batch256_instance_is_the_batch_member():
    """One instance generated alone equals the same member of the batch
    (same seed stream), and instance 168 is the 277^2 13-point problem the
    freeze-tolerance tests use."""
    batch = I.batch256(count=3)
    for i in range(3):
        a, b = batch[i], I.batch256_instance(i)
        assert (a.nx, a.ny, a.alpha, a.kappa, a.sigma) == (b.nx, b.ny, b.alpha, b.kappa, b.sigma)
        np.testing.assert_array_equal(a.cells, b.cells)
        np.testing.assert_array_equal(a.y, b.y)
    p = I.batch256_instance(168)
    assert (p.nx, p.ny, p.alpha) == (277, 277, 2)
