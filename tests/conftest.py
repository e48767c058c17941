import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# Stencil directions of the lattice message planes, as documented in
# include/gabp.h: plane d at (x, y) holds the message INTO (x, y) FROM
# (x + dx, y + dy); the opposite direction of d is d ^ 1.
DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1), (2, 0), (-2, 0), (0, 2), (0, -2),
        (1, 1), (-1, -1), (1, -1), (-1, 1)]


def n_dirs(alpha):
    return 4 if alpha == 1 else 12


def _wrap(v, n, periodic):
    if periodic:
        return v % n, True
    return v, (0 <= v < n)


def plane_slot_map(prob, graph):
    """For every (d, y, x) slot with an in-grid sender, the oracle CSR slot.

    Returns (d_idx, y_idx, x_idx, e_idx) arrays; slots without a sender are
    absent (their messages are identically zero).
    """
    from paper_2404_12968_amd.inputs import BC_PERIODIC
    nx, ny = prob.nx, prob.ny
    px, py = prob.bc_x == BC_PERIODIC, prob.bc_y == BC_PERIODIC
    out_d, out_y, out_x, out_e = [], [], [], []
    ys, xs = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i = (ys * nx + xs).ravel()
    key_all = graph.rows * graph.n + graph.col
    for d in range(n_dirs(prob.alpha)):
        dx, dy = DIRS[d]
        sx = xs + dx
        sy = ys + dy
        if px:
            sx = sx % nx
            okx = np.ones_like(sx, dtype=bool)
        else:
            okx = (sx >= 0) & (sx < nx)
        if py:
            sy = sy % ny
            oky = np.ones_like(sy, dtype=bool)
        else:
            oky = (sy >= 0) & (sy < ny)
        ok = (okx & oky).ravel()
        j = (sy * nx + sx).ravel()
        key = i[ok] * graph.n + j[ok]
        e = np.searchsorted(key_all, key)
        assert np.all(key_all[e] == key), "lattice slot without a graph edge"
        out_d.append(np.full(ok.sum(), d))
        out_y.append(ys.ravel()[ok])
        out_x.append(xs.ravel()[ok])
        out_e.append(e)
    return (np.concatenate(out_d), np.concatenate(out_y), np.concatenate(out_x),
            np.concatenate(out_e))


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.lib()
    return O
