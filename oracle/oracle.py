"""ctypes binding of the CPU oracle (test infrastructure only).

Thin marshalling of numpy arrays into oracle/liboracle.so.  Every function
mirrors one C entry point of sgmres_oracle.c, which cites the paper passage it
implements.  Builds the library with gcc on first use if it is missing.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "OK", "NOT_CONVERGED", "FLAG_KAPPA_TRUNC", "FLAG_BREAKDOWN", "KAPPA_MAX",
    "philox4x32_10", "sketch_pattern", "sketch_apply", "sketch_dense", "csr_spmv",
    "csr_transpose", "residual", "arnoldi_cycle", "sketched_lsq", "basis_combine",
    "sgmres_solve", "sgmres_solve_transposed", "dense_solve_gradient", "lib",
    "chebyshev_cycle", "sgmres_solve_chebyshev", "set_threads", "get_threads", "ritz_values",
    "chebyshev_box",
]

OK = 0
NOT_CONVERGED = 1
FLAG_KAPPA_TRUNC = 1
FLAG_BREAKDOWN = 2
KAPPA_MAX = 1e14  # Section 3.4: kappa_2(AB) <= 1e14 suffices in FP64

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_c = ctypes


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from .build_oracle import build

            build()
        L = ctypes.CDLL(path)
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_sketch_pattern.argtypes = [_c.c_uint64, _c.c_uint32, _c.c_int64, _c.c_int, _c.c_int, _i32p, _i8p]
        L.oracle_sketch_pattern.restype = None
        L.oracle_sketch_apply.argtypes = [_c.c_int64, _f64p, _c.c_uint64, _c.c_uint32, _c.c_int, _c.c_int, _f64p]
        L.oracle_sketch_apply.restype = _c.c_int
        L.oracle_csr_spmv.argtypes = [_c.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.oracle_csr_spmv.restype = None
        L.oracle_csr_transpose.argtypes = [_c.c_int64, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]
        L.oracle_csr_transpose.restype = _c.c_int
        L.oracle_residual.argtypes = [_c.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p]
        L.oracle_residual.restype = _c.c_double
        L.oracle_arnoldi_cycle.argtypes = [
            _c.c_int64, _i32p, _i32p, _f64p, _f64p, _c.c_int, _c.c_int, _c.c_int, _c.c_int,
            _c.c_uint64, _c.c_uint32, _c.c_int, _f64p, _f64p, _f64p, _f64p, _f64p,
            _c.POINTER(_c.c_int),
        ]
        L.oracle_arnoldi_cycle.restype = _c.c_int
        L.oracle_sketched_lsq.argtypes = [
            _c.c_int, _c.c_int, _f64p, _f64p, _c.c_double, _f64p, _f64p,
            _c.POINTER(_c.c_int), _c.POINTER(_c.c_double), _c.POINTER(_c.c_double),
            _c.POINTER(_c.c_int),
        ]
        L.oracle_sketched_lsq.restype = _c.c_int
        L.oracle_basis_combine.argtypes = [_c.c_int64, _c.c_int, _f64p, _f64p, _f64p]
        L.oracle_basis_combine.restype = None
        L.oracle_chebyshev_cycle.argtypes = [
            _c.c_int64, _i32p, _i32p, _f64p, _f64p, _c.c_int, _c.c_int, _c.c_int, _c.c_uint64, _c.c_uint32,
            _c.c_double, _c.c_double, _c.c_double, _f64p, _f64p, _f64p, _f64p, _f64p,
        ]
        L.oracle_chebyshev_cycle.restype = _c.c_int
        L.oracle_sgmres_solve_basis.argtypes = [
            _c.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p, _c.c_int, _c.c_int, _c.c_int,
            _c.c_int, _c.c_uint64, _c.c_double, _c.c_int, _c.c_double, _c.c_int, _c.c_double, _c.c_double,
            _c.c_double, _f64p,
        ]
        L.oracle_sgmres_solve_basis.restype = _c.c_int
        for name in ("oracle_sgmres_solve", "oracle_sgmres_solve_transposed"):
            fn = getattr(L, name)
            fn.argtypes = [
                _c.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p, _c.c_int, _c.c_int, _c.c_int,
                _c.c_int, _c.c_uint64, _c.c_double, _c.c_int, _c.c_double, _f64p,
            ]
            fn.restype = _c.c_int
        L.oracle_set_threads.argtypes = [_c.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_get_threads.argtypes = []
        L.oracle_get_threads.restype = _c.c_int
        _LIB = L
    return _LIB


def set_threads(t: int) -> None:
    """OpenMP threads of the row loops and fixed-chunk sums (bits do not depend on it)."""
    lib().oracle_set_threads(int(t))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def _csr(A):
    return (
        np.ascontiguousarray(A.row_ptr, dtype=np.int32),
        np.ascontiguousarray(A.col_idx, dtype=np.int32),
        np.ascontiguousarray(A.val, dtype=np.float64),
    )


def philox4x32_10(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def sketch_pattern(seed: int, cycle: int, i0: int, count: int, s: int, zeta: int):
    """Rows (int32[count, zeta]) and signs (int8[count, zeta]) of columns i0..i0+count-1."""
    rows = np.zeros((count, zeta), np.int32)
    signs = np.zeros((count, zeta), np.int8)
    L = lib()
    r1 = np.zeros(zeta, np.int32)
    s1 = np.zeros(zeta, np.int8)
    for q in range(count):
        L.oracle_sketch_pattern(seed, cycle, i0 + q, s, zeta, r1, s1)
        rows[q] = r1
        signs[q] = s1
    return rows, signs


def sketch_apply(v, seed: int, cycle: int, s: int, zeta: int) -> np.ndarray:
    v = np.ascontiguousarray(v, np.float64)
    g = np.zeros(s, np.float64)
    rc = lib().oracle_sketch_apply(v.size, v, seed, cycle, s, zeta, g)
    if rc != OK:
        raise ValueError(f"oracle_sketch_apply rc={rc}")
    return g


def sketch_dense(n: int, seed: int, cycle: int, s: int, zeta: int) -> np.ndarray:
    """The s x n sketch matrix as a dense array (tiny n only)."""
    rows, signs = sketch_pattern(seed, cycle, 0, n, s, zeta)
    S = np.zeros((s, n))
    for i in range(n):
        S[rows[i], i] = signs[i]
    return S / np.sqrt(zeta)


def csr_spmv(A, x) -> np.ndarray:
    rp, ci, v = _csr(A)
    y = np.zeros(A.n, np.float64)
    lib().oracle_csr_spmv(A.n, rp, ci, v, np.ascontiguousarray(x, np.float64), y)
    return y


def csr_transpose(A):
    from synth import CSR

    rp, ci, v = _csr(A)
    trp = np.zeros(A.n + 1, np.int32)
    tci = np.zeros(max(A.nnz, 1), np.int32)
    tv = np.zeros(max(A.nnz, 1), np.float64)
    rc = lib().oracle_csr_transpose(A.n, rp, ci, v, trp, tci, tv)
    if rc != OK:
        raise MemoryError
    return CSR(n=A.n, row_ptr=trp, col_idx=tci[: A.nnz], val=tv[: A.nnz])


def residual(A, f, x):
    rp, ci, v = _csr(A)
    r = np.zeros(A.n, np.float64)
    nrm = lib().oracle_residual(
        A.n, rp, ci, v, np.ascontiguousarray(f, np.float64), np.ascontiguousarray(x, np.float64), r
    )
    return r, nrm


def arnoldi_cycle(A, r, d: int, k: int, s: int, zeta: int, seed: int, cycle: int = 0, passes: int = 2):
    """One cycle of basis generation + sketching; returns a dict of arrays."""
    rp, ci, v = _csr(A)
    n = A.n
    B = np.zeros((d, n))  # row q = column q of the column-major n x d basis
    SB = np.zeros((d, s))
    SAB = np.zeros((d, s))
    H = np.zeros((d, k + 1))
    g = np.zeros(s)
    flags = ctypes.c_int(0)
    dc = lib().oracle_arnoldi_cycle(
        n, rp, ci, v, np.ascontiguousarray(r, np.float64), d, k, s, zeta, seed, cycle, passes,
        B, SB, SAB, H, g, ctypes.byref(flags),
    )
    if dc < 0:
        raise ValueError(f"oracle_arnoldi_cycle rc={dc}")
    return dict(B=B.T.copy(), SB=SB.T.copy(), SAB=SAB.T.copy(), H=H.T.copy(), g=g, dc=dc, flags=flags.value)


def chebyshev_cycle(A, r, d: int, s: int, zeta: int, seed: int, cycle: int, c: float, dx: float, dy: float):
    """One Chebyshev-basis cycle (Section 4.4) + sketching; returns a dict with the
    normalised basis B (n x d), SB, SAB (s x d), the raw norms nrm (d) and g."""
    rp, ci, v = _csr(A)
    n = A.n
    B = np.zeros((d, n))
    SB = np.zeros((d, s))
    SAB = np.zeros((d, s))
    nrm = np.zeros(d)
    g = np.zeros(s)
    rc = lib().oracle_chebyshev_cycle(n, rp, ci, v, np.ascontiguousarray(r, np.float64), d, s, zeta, seed, cycle,
                                      c, dx, dy, B, SB, SAB, nrm, g)
    if rc < 0:
        raise ValueError(f"oracle_chebyshev_cycle rc={rc}")
    return dict(B=B.T.copy(), SB=SB.T.copy(), SAB=SAB.T.copy(), nrm=nrm, g=g)


def sketched_lsq(SAB, g, kappa_max: float = KAPPA_MAX):
    """Householder sketched LS on SAB (s x dc) and g; returns a dict."""
    SAB = np.asarray(SAB, np.float64)
    s, dc = SAB.shape
    C = np.ascontiguousarray(SAB.T)  # column-major storage
    gg = np.array(g, np.float64, copy=True)
    y = np.zeros(max(dc, 1))
    tau = np.zeros(max(dc, 1))
    d_eff = ctypes.c_int(0)
    rest = ctypes.c_double(0)
    kap = ctypes.c_double(0)
    flags = ctypes.c_int(0)
    rc = lib().oracle_sketched_lsq(
        s, dc, C, gg, kappa_max, y, tau, ctypes.byref(d_eff), ctypes.byref(rest), ctypes.byref(kap),
        ctypes.byref(flags),
    )
    if rc != OK:
        raise ValueError(f"oracle_sketched_lsq rc={rc}")
    de = d_eff.value
    return dict(
        y=y[:de].copy(), d_eff=de, rest=rest.value, kappa=kap.value, flags=flags.value,
        T=np.triu(C.T[:dc, :dc]), QTg=gg, tau=tau[:dc].copy(),
    )


def basis_combine(B, y, x) -> np.ndarray:
    B = np.asarray(B, np.float64)
    n = B.shape[0]
    d_eff = len(y)
    Bc = np.ascontiguousarray(B[:, :d_eff].T) if d_eff else np.zeros(1)
    out = np.array(x, np.float64, copy=True)
    lib().oracle_basis_combine(n, d_eff, Bc, np.ascontiguousarray(y, np.float64) if d_eff else np.zeros(1), out)
    return out


def _solve(name, A, b, x0, d, k, s, zeta, seed, tol, restarts, kappa_max):
    rp, ci, v = _csr(A)
    x = np.zeros(A.n) if x0 is None else np.array(x0, np.float64, copy=True)
    info = np.zeros(8)
    rc = getattr(lib(), name)(
        A.n, rp, ci, v, np.ascontiguousarray(b, np.float64), x, d, k, s, zeta, seed, tol, restarts,
        kappa_max, info,
    )
    return rc, x, dict(
        cycles=int(info[0]), steps=int(info[1]), d_eff_last=int(info[2]), flags=int(info[3]),
        relres=float(info[4]), rest_est=float(info[5]), kappa_est=float(info[6]),
    )


def sgmres_solve(A, b, x0=None, d=40, k=2, s=None, zeta=8, seed=0, tol=1e-10, restarts=100,
                 kappa_max=KAPPA_MAX):
    """Restarted sGMRES on A x = b.  Returns (rc, x, info)."""
    s = 2 * d if s is None else s
    return _solve("oracle_sgmres_solve", A, b, x0, d, k, s, zeta, seed, tol, restarts, kappa_max)


def sgmres_solve_chebyshev(A, b, box, x0=None, d=40, s=None, zeta=8, seed=0, tol=1e-10, restarts=100,
                           kappa_max=KAPPA_MAX):
    """Restarted sGMRES with the Chebyshev basis for box = (c, dx, dy).  Returns (rc, x, info)."""
    s = 2 * d if s is None else s
    rp, ci, v = _csr(A)
    x = np.zeros(A.n) if x0 is None else np.array(x0, np.float64, copy=True)
    info = np.zeros(8)
    c, dx, dy = (float(t) for t in box)
    rc = lib().oracle_sgmres_solve_basis(
        A.n, rp, ci, v, np.ascontiguousarray(b, np.float64), x, d, 1, s, zeta, seed, tol, restarts, kappa_max,
        1, c, dx, dy, info,
    )
    return rc, x, dict(
        cycles=int(info[0]), steps=int(info[1]), d_eff_last=int(info[2]), flags=int(info[3]),
        relres=float(info[4]), rest_est=float(info[5]), kappa_est=float(info[6]),
    )


def ritz_values(A, r, m: int):
    """Ritz values of an m-step Arnoldi process on A from r (Section 4.4: a few
    Arnoldi iterations estimate the spectrum): m + 1 steps of the oracle's
    Arnoldi with a full window, the leading m x m block of its Hessenberg
    matrix (the leading dc x dc block when the basis stops at dc columns), and
    that block's eigenvalues (numpy's dense eigenvalue routine)."""
    d, k = m + 1, m
    s = max(d + 1, 16)
    out = arnoldi_cycle(A, r, d=d, k=k, s=s, zeta=8, seed=0, cycle=0)
    H = out["H"]  # (k + 1) x d: H[a, j] = coefficient of window entry a (newest first), H[k, j] = nu_j
    me = min(m, int(out["dc"]))
    Hm = np.zeros((me, me))
    for j in range(me):
        for a in range(j + 1):
            Hm[j - a, j] = H[a, j]
        if j + 1 < me:
            Hm[j + 1, j] = H[k, j]
    return np.linalg.eigvals(Hm)


def chebyshev_box(A, r, m: int, margin: float = 0.1):
    """The spectral box (c, dx, dy) for the Chebyshev basis from the Ritz values
    of ritz_values(A, r, m): their bounding rectangle [c +- dx] x [+-dy], both
    half-widths widened by the fraction margin (a reading: the paper leaves the
    fit of the region to the estimated spectrum open)."""
    th = ritz_values(A, r, m)
    xmin, xmax = float(th.real.min()), float(th.real.max())
    ymax = float(np.abs(th.imag).max())
    return 0.5 * (xmin + xmax), (1.0 + margin) * 0.5 * (xmax - xmin), (1.0 + margin) * ymax


def sgmres_solve_transposed(A, b, x0=None, d=40, k=2, s=None, zeta=8, seed=0, tol=1e-10,
                            restarts=100, kappa_max=KAPPA_MAX):
    """Restarted sGMRES on A^T x = b.  Returns (rc, x, info)."""
    s = 2 * d if s is None else s
    return _solve("oracle_sgmres_solve_transposed", A, b, x0, d, k, s, zeta, seed, tol, restarts, kappa_max)


def dense_solve_gradient(A, b, xt):
    """Loss L = |x - xt|^2 with x = A^{-1} b, in dense FP64 (numpy.linalg.solve).

    Adjoint: A^T lam = dL/dx = 2 (x - xt); dL/db = lam; dL/dA_ij = -lam_i x_j,
    returned on A's stored pattern (same order as A.val).  Returns
    (x, L, dL/db, dL/dval)."""
    D = A.to_dense()
    x = np.linalg.solve(D, np.asarray(b, np.float64))
    diff = x - xt
    L = float(diff @ diff)
    lam = np.linalg.solve(D.T, 2.0 * diff)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    gval = -lam[rows] * x[A.col_idx]
    return x, L, lam, gval
