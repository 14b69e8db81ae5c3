"""Seeded synthetic operators and right-hand sides.

Everything here is deterministic given its seed.  The operators stand in for the
paper's test matrices (Section 7.1: a nonsymmetric SuiteSparse system of order
about 9.2e5 and a 2D Laplacian of order 1e6), which are not available here:

* ``convection_diffusion`` -- 5-point central-difference discretisation of
  -Laplace(u) + beta . grad(u) on the unit square with homogeneous Dirichlet
  boundary, scaled by h^2.  beta = 0 gives the 2D Laplacian class of Section 7.1.3;
  beta != 0 gives a nonsymmetric operator like the one of Section 7.1.2.
* ``random_dominant`` -- random sparse nonsymmetric rows (diagonal plus distinct
  random off-diagonal columns with N(0,1) values), made strictly diagonally
  dominant.

CSR arrays use int32 row pointers / column indices (sorted within each row) and
float64 values.
"""

from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass
class CSR:
    """Square sparse matrix in compressed sparse row form (host arrays)."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.n, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        out[rows, self.col_idx] = self.val
        return out


def _csr_from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    return CSR(
        n=n,
        row_ptr=row_ptr.astype(np.int32),
        col_idx=cols.astype(np.int32),
        val=np.ascontiguousarray(vals, dtype=np.float64),
    )


def convection_diffusion(N: int, beta=(0.0, 0.0)) -> CSR:
    """5-point convection-diffusion operator on an N x N interior grid.

    Unknown (ix, iy) has index ix + N*iy (x fastest).  With h = 1/(N+1) and the
    equation multiplied by h^2, row entries are: diagonal 4; west -1 - bx*h/2;
    east -1 + bx*h/2; south -1 - by*h/2; north -1 + by*h/2.  nnz = 5N^2 - 4N.
    """
    bx, by = float(beta[0]), float(beta[1])
    h = 1.0 / (N + 1)
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    ix = idx % N
    iy = idx // N
    parts_r, parts_c, parts_v = [idx], [idx], [np.full(n, 4.0)]
    stencil = [
        (ix > 0, -1, -1.0 - bx * h / 2),  # west
        (ix < N - 1, +1, -1.0 + bx * h / 2),  # east
        (iy > 0, -N, -1.0 - by * h / 2),  # south
        (iy < N - 1, +N, -1.0 + by * h / 2),  # north
    ]
    for mask, off, coef in stencil:
        r = idx[mask]
        parts_r.append(r)
        parts_c.append(r + off)
        parts_v.append(np.full(r.size, coef))
    return _csr_from_coo(n, np.concatenate(parts_r), np.concatenate(parts_c), np.concatenate(parts_v))


def random_dominant(n: int, offdiag: int = 6, seed=0, dominance: float = 1.2) -> CSR:
    """Random sparse nonsymmetric matrix, strictly diagonally dominant by rows.

    Each row holds the diagonal plus ``offdiag`` distinct off-diagonal columns
    drawn uniformly; off-diagonal values are N(0,1); the diagonal is
    ``dominance`` times the row's off-diagonal absolute sum.
    """
    rng = np.random.default_rng(seed)
    m = min(offdiag, n - 1)
    if m <= 0:
        return _csr_from_coo(n, np.arange(n), np.arange(n), np.ones(n))
    # distinct off-diagonal columns per row: draw from [0, n-1) and shift past i;
    # redraw rows with duplicates until each row has m distinct columns.
    cols = rng.integers(0, n - 1, size=(n, m), dtype=np.int64)
    while True:
        s = np.sort(cols, axis=1)
        dup = np.any(s[:, 1:] == s[:, :-1], axis=1) if m > 1 else np.zeros(n, bool)
        if not dup.any():
            break
        cols[dup] = rng.integers(0, n - 1, size=(int(dup.sum()), m), dtype=np.int64)
    ar = np.arange(n, dtype=np.int64)
    cols = cols + (cols >= ar[:, None])  # skip the diagonal
    vals = rng.standard_normal(n * m).reshape(n, m)
    diag = np.zeros(n)
    for t in range(m):  # row sums in column order
        diag += np.abs(vals[:, t])
    diag *= dominance
    diag[diag == 0] = 1.0
    # every row holds m + 1 distinct columns: sort within rows (CSR order)
    allc = np.concatenate([cols, ar[:, None]], axis=1)
    allv = np.concatenate([vals, diag[:, None]], axis=1)
    order = np.argsort(allc, axis=1, kind="stable")
    allc = np.take_along_axis(allc, order, axis=1)
    allv = np.take_along_axis(allv, order, axis=1)
    if n * (m + 1) >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    return CSR(
        n=n,
        row_ptr=(np.arange(n + 1, dtype=np.int64) * (m + 1)).astype(np.int32),
        col_idx=allc.reshape(-1).astype(np.int32),
        val=np.ascontiguousarray(allv.reshape(-1), dtype=np.float64),
    )


def diagonal(values) -> CSR:
    v = np.asarray(values, dtype=np.float64)
    n = v.size
    ar = np.arange(n)
    return _csr_from_coo(n, ar, ar, v)


def rhs(n: int, seed=0) -> np.ndarray:
    """Right-hand side b ~ N(0, I) from numpy's default generator."""
    return np.random.default_rng(seed).standard_normal(n)


def batched_random_systems(count: int = 256, lo: int = 16384, hi: int = 262144, seed: int = 4):
    """Sizes and generator seeds of the many-systems workload (uneven n)."""
    sizes = np.random.default_rng(seed).integers(lo, hi, endpoint=True, size=count)
    return [(int(n_i), [seed, i]) for i, n_i in enumerate(sizes)]


def batch_workload(count: int = 256, lo: int = 16384, hi: int = 262144, seed: int = 4):
    """The many-systems workload: system i is random_dominant(n_i, 6 off-diagonals,
    seed [seed, i]) with b_i ~ N(0, I) from default_rng([0, i]).  Returns a list of
    (A_i, b_i)."""
    return [(random_dominant(n_i, offdiag=6, seed=sd), rhs(n_i, [0, i]))
            for i, (n_i, sd) in enumerate(batched_random_systems(count, lo, hi, seed))]


def block_rhs_workload(n: int = 1 << 20, nrhs: int = 32, seed: int = 2):
    """One random_dominant(n, 6 off-diagonals, seed) matrix with nrhs right-hand
    sides b_j ~ N(0, I) from default_rng([seed, j])."""
    return random_dominant(n, offdiag=6, seed=seed), [rhs(n, [seed, j]) for j in range(nrhs)]


# Named workloads: operator recipe + solver parameters.
WORKLOADS = {
    # small one-cycle case: n = 4096, d = 40, k = 2, s = 80
    "cd64": dict(N=64, beta=(10.0, 10.0), d=40, k=2, s=80, zeta=8, seed=0, tol=0.0, restarts=0),
    # full-size FP64 case: n = 1,048,576, d = 200, k = 4, s = 400, restarted to 1e-10
    "cd1024": dict(N=1024, beta=(50.0, 20.0), d=200, k=4, s=400, zeta=8, seed=0, tol=1e-10, restarts=1000),
    # mixed-precision case: n = 4,194,304
    "cd2048": dict(N=2048, beta=(50.0, 20.0), d=200, k=4, s=400, zeta=8, seed=0, tol=1e-10, restarts=1000),
    # differentiable-solve finite-difference check: n = 1024
    "cd32": dict(N=32, beta=(50.0, 20.0), d=200, k=4, s=400, zeta=8, seed=0, tol=1e-10, restarts=1000),
    # random sparse nonsymmetric, well conditioned (diagonal dominance 1.2):
    # n = 1,048,576, 7 nonzeros per row, the batched-workload parameters
    "rd1m": dict(rand_n=1 << 20, offdiag=6, mat_seed=4, d=100, k=2, s=200, zeta=8, seed=0, tol=1e-10,
                 restarts=1000),
}


def workload(name: str):
    """Return (A, b, params) for a named workload."""
    p = dict(WORKLOADS[name])
    if "rand_n" in p:
        A = random_dominant(p.pop("rand_n"), offdiag=p.pop("offdiag"), seed=p.pop("mat_seed"))
    else:
        A = convection_diffusion(p.pop("N"), p.pop("beta"))
    b = rhs(A.n, 0)
    return A, b, p
