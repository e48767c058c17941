"""CPU oracle for lattice GMRF data assimilation by re-weighted Gaussian BP.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the GPU library or its binding.
It shares no code with the GPU path; only the seeded input generators are
common to both.

Contents, each following the paper:

* ``laplacian_1d`` / ``precision``: the finite-difference operator
  L = kappa^2 I - Delta_h (Appendix "Details on the Finite Difference
  Discretisation", the discretised-operator equation) on a 2-D grid, and the
  prior precision Q = tau L^alpha formed by sparse matrix products
  (Section "Derivation of the Factor Graph": P = gamma L^T L, sparse when
  alpha/2 is an integer).  Boundary readings: periodic and Dirichlet as in the
  appendix; Neumann (zero flux, not in the paper) as the graph Laplacian of
  the path.
* ``observation_terms``: Gaussian point likelihood folded into the node
  factor (Section "Including Observations"); unobserved cells add nothing
  (the "very large z" read as z = infinity).
* ``FactorGraph``: nodes and an edge wherever A_ij != 0 (Section
  "Derivation of the Factor Graph"), CSR with a reverse-edge index.
* ``OracleGaBP``: the flooding, damped, re-weighted iteration of Algorithms
  1 and 2 (inner procedure) in FP64, run by ``gabp_oracle.c``; marginals
  (Compute Marginal); the FP64 residual; the paper's early-stop statistic.
* ``direct_solve``: the exact posterior mean A^{-1} b by sparse LU, which the
  method reaches at convergence.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gabp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libgabp_oracle.so")

BC_NEUMANN, BC_PERIODIC, BC_DIRICHLET = 0, 1, 2
STATUS_OK, STATUS_DIVERGED = 0, 4


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, IEEE, no fast-math) and OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        d = ctypes.c_double
        L.oracle_gabp_iterate.argtypes = [i64, P, P, P, P, P, P, d, d, i64, P, P, P]
        L.oracle_gabp_iterate.restype = ctypes.c_int
        L.oracle_beliefs.argtypes = [i64, P, P, P, d, P, P, P, P]
        L.oracle_beliefs.restype = None
        L.oracle_posterior.argtypes = [i64, P, P, P, d, P, P, P, P]
        L.oracle_posterior.restype = None
        L.oracle_residual.argtypes = [i64, P, P, P, P, P, P, P]
        L.oracle_residual.restype = None
        L.oracle_abs_change.argtypes = [i64, P, P, P, P]
        L.oracle_abs_change.restype = d
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


# --------------------------------------------------------------------------
# prior precision by sparse assembly
# --------------------------------------------------------------------------

def laplacian_1d(n: int, bc: int) -> sp.csr_matrix:
    """-d^2/dx^2 at unit spacing as an n x n sparse matrix.

    Periodic: the cycle's graph Laplacian (ghost points wrap).  Dirichlet: the
    boundary values are zero and removed, so every row keeps the full
    diagonal 2.  Neumann (reading): zero flux, the path's graph Laplacian.
    """
    if n == 1:
        return sp.csr_matrix((1, 1)) if bc != BC_DIRICHLET else sp.csr_matrix(np.array([[2.0]]))
    off = -np.ones(n - 1)
    if bc == BC_PERIODIC:
        if n < 3:
            raise ValueError("periodic axis needs at least 3 points")
        main = 2.0 * np.ones(n)
        m = sp.diags([off, main, off], [-1, 0, 1], shape=(n, n), format="lil")
        m[0, n - 1] += -1.0
        m[n - 1, 0] += -1.0
        return m.tocsr()
    if bc == BC_DIRICHLET:
        main = 2.0 * np.ones(n)
    else:
        main = 2.0 * np.ones(n)
        main[0] = main[-1] = 1.0
    return sp.diags([off, main, off], [-1, 0, 1], shape=(n, n), format="csr")


def operator_L(nx: int, ny: int, kappa: float, hx: float = 1.0, hy: float = 1.0,
               bc_x: int = BC_NEUMANN, bc_y: int = BC_NEUMANN) -> sp.csr_matrix:
    """L = kappa^2 I - Delta_h on the row-major grid (index y * nx + x)."""
    gx = laplacian_1d(nx, bc_x) / (hx * hx)
    gy = laplacian_1d(ny, bc_y) / (hy * hy)
    ix = sp.identity(nx, format="csr")
    iy = sp.identity(ny, format="csr")
    L = kappa * kappa * sp.identity(nx * ny, format="csr") + sp.kron(iy, gx) + sp.kron(gy, ix)
    return sp.csr_matrix(L)


def precision(nx: int, ny: int, alpha: int, kappa: float, tau: float = 1.0,
              hx: float = 1.0, hy: float = 1.0, bc_x: int = BC_NEUMANN,
              bc_y: int = BC_NEUMANN) -> sp.csr_matrix:
    """Prior precision Q = tau * L^alpha by sparse matrix products."""
    if alpha not in (1, 2):
        raise ValueError("alpha must be 1 or 2")
    L = operator_L(nx, ny, kappa, hx, hy, bc_x, bc_y)
    Q = L if alpha == 1 else (L @ L)
    Q = sp.csr_matrix(tau * Q)
    Q.sum_duplicates()
    Q.eliminate_zeros()
    Q.sort_indices()
    return Q


def observation_terms(n: int, cells: np.ndarray, y: np.ndarray, sigma: float,
                      var: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Per-node observation precision p_i = sum 1/s^2 and information h_i = sum y/s^2.

    Several observations of one cell add (product of their likelihoods).
    """
    cells = np.asarray(cells, dtype=np.int64)
    y = np.asarray(y, dtype=np.float64)
    w = (1.0 / np.asarray(var, dtype=np.float64)) if var is not None else \
        np.full(cells.size, 1.0 / (sigma * sigma))
    p = np.bincount(cells, weights=w, minlength=n).astype(np.float64)
    h = np.bincount(cells, weights=w * y, minlength=n).astype(np.float64)
    return p, h


def posterior_system(prob, prior_mean: Optional[np.ndarray] = None):
    """(A, b) with A = Q + diag(p) and b = h (+ Q f_b) for a Problem."""
    Q = precision(prob.nx, prob.ny, prob.alpha, prob.kappa, prob.tau, prob.hx, prob.hy,
                  prob.bc_x, prob.bc_y)
    p, h = observation_terms(prob.n, prob.cells, prob.y, prob.sigma, prob.var)
    A = sp.csr_matrix(Q + sp.diags(p))
    A.sort_indices()
    b = h.copy()
    if prior_mean is not None:
        b = b + Q @ np.asarray(prior_mean, dtype=np.float64).reshape(-1)
    return A, b


def direct_solve(A: sp.spmatrix, b: np.ndarray) -> np.ndarray:
    """Exact posterior mean A^{-1} b by sparse LU (scipy's SuperLU)."""
    return spla.splu(sp.csc_matrix(A)).solve(np.asarray(b, dtype=np.float64))


def full_coverage_mean(nx: int, ny: int, alpha: int, kappa: float, tau: float, p: float,
                       yv: np.ndarray, bc_x: int = BC_NEUMANN, bc_y: int = BC_NEUMANN,
                       hx: float = 1.0, hy: float = 1.0) -> np.ndarray:
    """Exact posterior mean when every cell is observed once with precision p.

    A = Q + p I and Q = tau (kappa^2 I + G_x/hx^2 + G_y/hy^2)^alpha share the
    eigenvectors of the 1-D Laplacians G: Fourier modes on a periodic axis
    (eigenvalues 4 sin^2(pi k / n)) and the DCT-II basis on a zero-flux axis
    (4 sin^2(pi k / 2n)).  So mu = V [p V^T y / (tau (kappa^2 + lambda)^alpha
    + p)], one separable transform per axis (FFT or orthonormal DCT-II).
    Returns mu as [ny, nx]."""
    import scipy.fft as sfft
    yv = np.asarray(yv, dtype=np.float64).reshape(ny, nx)

    def fwd(a, axis, bc):
        if bc == BC_PERIODIC:
            return np.fft.fft(a, axis=axis)
        if bc == BC_NEUMANN:
            return sfft.dct(a, type=2, norm="ortho", axis=axis)
        raise ValueError("closed form covers periodic and zero-flux axes")

    def inv(a, axis, bc):
        if bc == BC_PERIODIC:
            return np.fft.ifft(a, axis=axis)
        return sfft.idct(a, type=2, norm="ortho", axis=axis)

    def eig(n, bc, h):
        k = np.arange(n)
        arg = np.pi * k / n if bc == BC_PERIODIC else np.pi * k / (2 * n)
        return 4.0 * np.sin(arg) ** 2 / (h * h)

    lam = eig(nx, bc_x, hx)[None, :] + eig(ny, bc_y, hy)[:, None]
    yh = fwd(fwd(yv.astype(np.complex128) if BC_PERIODIC in (bc_x, bc_y) else yv, 1, bc_x),
             0, bc_y)
    mh = p * yh / (tau * (kappa * kappa + lam) ** alpha + p)
    mu = inv(inv(mh, 0, bc_y), 1, bc_x)
    return np.real(mu)


# --------------------------------------------------------------------------
# factor graph and message passing
# --------------------------------------------------------------------------

class FactorGraph:
    """Pairwise factor graph of a symmetric matrix A.

    Node factor of i: A_ii and b_i.  Edge (i, j) wherever A_ij != 0, i != j.
    CSR row i lists the neighbours j; ``rev[e]`` is the slot of (j, i).
    """

    def __init__(self, A: sp.spmatrix, b: np.ndarray):
        A = sp.csr_matrix(A, dtype=np.float64)
        n = A.shape[0]
        self.n = n
        self.adiag = np.ascontiguousarray(A.diagonal().astype(np.float64))
        off = sp.csr_matrix(A - sp.diags(A.diagonal()))
        off.eliminate_zeros()
        off.sort_indices()
        self.row_ptr = np.ascontiguousarray(off.indptr.astype(np.int64))
        self.col = np.ascontiguousarray(off.indices.astype(np.int64))
        self.aoff = np.ascontiguousarray(off.data.astype(np.float64))
        rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(self.row_ptr))
        self.rows = rows
        key = rows * n + self.col
        rkey = self.col * n + rows
        rev = np.searchsorted(key, rkey)
        if rev.size and (np.any(rev >= key.size) or np.any(key[np.minimum(rev, key.size - 1)] != rkey)):
            raise ValueError("matrix is not structurally symmetric")
        self.rev = np.ascontiguousarray(rev.astype(np.int64))
        if not np.allclose(self.aoff[self.rev], self.aoff, rtol=1e-13, atol=0):
            raise ValueError("matrix is not symmetric")
        # exact symmetry (the products forming Q may round the two halves apart)
        self.aoff = np.ascontiguousarray(0.5 * (self.aoff + self.aoff[self.rev]))
        self.b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
        self.nnz = int(self.col.size)


class OracleGaBP:
    """FP64 flooding GaBP state: messages m^t on every directed edge.

    ``lam[e]``, ``th[e]`` for slot e = (i, j) of the CSR hold the message INTO
    i FROM j.  Initial messages are zero unless given.
    """

    def __init__(self, graph: FactorGraph, c: float, lam0=None, th0=None):
        if c == 0:
            raise ValueError("c must be non-zero")
        self.g = graph
        self.c = float(c)
        self.lam = np.zeros(graph.nnz) if lam0 is None else np.array(lam0, dtype=np.float64)
        self.th = np.zeros(graph.nnz) if th0 is None else np.array(th0, dtype=np.float64)
        self.t = 0
        self.diverged_at = None
        self._ref_change = None
        self._prev = None

    @classmethod
    def from_problem(cls, prob, c: Optional[float] = None, prior_mean=None):
        A, b = posterior_system(prob, prior_mean)
        return cls(FactorGraph(A, b), prob.c if c is None else c)

    def iterate(self, iters: int, eta: float, keep_prev: bool = False) -> int:
        """Run ``iters`` flooding iterations with damping ``eta``.  Returns status."""
        g = self.g
        if keep_prev:
            self._prev = (self.lam.copy(), self.th.copy())
        done = ctypes.c_int64(0)
        st = lib().oracle_gabp_iterate(g.n, _p(g.row_ptr), _p(g.col), _p(g.aoff), _p(g.rev),
                                        _p(g.adiag), _p(g.b), self.c, float(eta), int(iters),
                                        _p(self.lam), _p(self.th), ctypes.byref(done))
        self.t += int(done.value)
        if st == STATUS_DIVERGED:
            self.diverged_at = self.t
        elif st != STATUS_OK:
            raise MemoryError("oracle allocation failed")
        return st

    def beliefs(self):
        g = self.g
        bl = np.empty(g.n)
        bt = np.empty(g.n)
        lib().oracle_beliefs(g.n, _p(g.row_ptr), _p(g.adiag), _p(g.b), self.c,
                             _p(self.lam), _p(self.th), _p(bl), _p(bt))
        return bl, bt

    def posterior(self):
        g = self.g
        mu = np.empty(g.n)
        var = np.empty(g.n)
        lib().oracle_posterior(g.n, _p(g.row_ptr), _p(g.adiag), _p(g.b), self.c,
                               _p(self.lam), _p(self.th), _p(mu), _p(var))
        return mu, var

    def residual(self, mu: Optional[np.ndarray] = None):
        """(relative, absolute) FP64 residual ||A mu - b||_2 (relative to ||b||_2)."""
        g = self.g
        if mu is None:
            mu, _ = self.posterior()
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        out = np.empty(2)
        lib().oracle_residual(g.n, _p(g.row_ptr), _p(g.col), _p(g.aoff), _p(g.adiag),
                              _p(g.b), _p(mu), _p(out))
        rel = out[0] / out[1] if out[1] > 0 else out[0]
        return float(rel), float(out[0])

    def solve(self, max_iters: int, eta: float, rel_tol: float, check_every: int = 10):
        """Iterate in chunks until the relative residual is <= rel_tol."""
        while self.t < max_iters:
            k = min(check_every, max_iters - self.t)
            st = self.iterate(k, eta)
            if st == STATUS_DIVERGED:
                return st, self.residual()[0]
            rel, _ = self.residual()
            if rel <= rel_tol:
                return STATUS_OK, rel
        return 5, self.residual()[0]

    def abs_change(self, lam_a, th_a, lam_b, th_b) -> float:
        """Sum over every directed edge of |lam_a - lam_b| + |th_a - th_b|."""
        return float(lib().oracle_abs_change(self.g.nnz, _p(np.ascontiguousarray(lam_a)),
                                             _p(np.ascontiguousarray(th_a)),
                                             _p(np.ascontiguousarray(lam_b)),
                                             _p(np.ascontiguousarray(th_b))))

    def early_stop_statistic(self, prev, m1, m2) -> float:
        """The paper's early-stopping statistic (Appendix A, Early Stop):
        mean|m^t - m^{t-1}| / mean|m^2 - m^1| for the current messages m^t,
        prev = m^{t-1} and m1, m2 the first two iterations, each a pair
        (lam, th).  Both components of every directed message are pooled in
        one mean (reading of "mean(abs(...))"); both means run over the same
        entries, so the ratio is that of the sums."""
        num = self.abs_change(self.lam, self.th, prev[0], prev[1])
        den = self.abs_change(m2[0], m2[1], m1[0], m1[1])
        return num / den
