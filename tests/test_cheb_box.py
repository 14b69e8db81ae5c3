"""Spectral box for the Chebyshev basis from a short Arnoldi pass (Section 4.4).

CPU tests: the oracle's Ritz values pinned to dense eigenvalues (numpy) where
they are exact (a Krylov space that is an invariant subspace) and to the
interlacing bounds of a symmetric matrix; the box's construction; and the
library's host Hessenberg eigenvalue routine against numpy on random
matrices.  The GPU tests are in tests/test_gpu_chebyshev.py.
"""

import ctypes
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth

PKG = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2111_00113_amd")
LIB = os.path.join(PKG, "libsgmres.so")


def csr_of(M):
    M = sp.csr_matrix(M)
    return synth.CSR(n=M.shape[0], row_ptr=M.indptr.astype(np.int32), col_idx=M.indices.astype(np.int32),
                     val=M.data.astype(np.float64))


def block_system(q=7, n=40, seed=3):
    """A = diag(A1, A2) with r supported on the first q coordinates: the Krylov
    space of r is an invariant subspace of dimension q, so the Arnoldi process
    stops after q columns and its Ritz values are exactly eig(A1)."""
    rng = np.random.default_rng(seed)
    A1 = rng.standard_normal((q, q)) + 3.0 * np.eye(q)
    Ad = np.zeros((n, n))
    Ad[:q, :q] = A1
    Ad[q:, q:] = rng.standard_normal((n - q, n - q))
    r = np.zeros(n)
    r[:q] = rng.standard_normal(q)
    return csr_of(Ad), r, np.linalg.eigvals(A1)


def nearest_gap(a, b):
    return max(min(abs(x - y) for x in a) for y in b)


def test_ritz_values_of_an_invariant_subspace_are_its_eigenvalues(orc):
    A, r, ev = block_system()
    th = orc.ritz_values(A, r, 12)
    assert len(th) == len(ev)
    assert nearest_gap(th, ev) <= 1e-12 * np.abs(ev).max()
    assert nearest_gap(ev, th) <= 1e-12 * np.abs(ev).max()


def test_ritz_values_of_a_symmetric_matrix_interlace(orc):
    # symmetric A: Ritz values are real and lie in [lambda_min, lambda_max]
    rng = np.random.default_rng(8)
    n = 300
    M = sp.random(n, n, density=0.02, random_state=4)
    S = (M + M.T).toarray() + np.diag(rng.uniform(1.0, 5.0, n))
    ev = np.linalg.eigvalsh(S)
    th = orc.ritz_values(csr_of(S), rng.standard_normal(n), 20)
    assert np.abs(th.imag).max() <= 1e-10 * np.abs(ev).max()
    assert th.real.min() >= ev[0] - 1e-10 and th.real.max() <= ev[-1] + 1e-10
    # the extreme Ritz values approach the extreme eigenvalues from inside
    assert th.real.max() >= ev[-1] - 0.2 * (ev[-1] - ev[0])


def test_box_is_the_widened_bounding_rectangle(orc):
    A, r, ev = block_system()
    c, dx, dy = orc.chebyshev_box(A, r, 12, margin=0.1)
    lo, hi, im = ev.real.min(), ev.real.max(), np.abs(ev.imag).max()
    assert np.isclose(c, 0.5 * (lo + hi), rtol=1e-12)
    assert np.isclose(dx, 1.1 * 0.5 * (hi - lo), rtol=1e-12)
    assert np.isclose(dy, 1.1 * im, rtol=1e-12)
    # every eigenvalue of the block lies inside the box
    assert np.all(np.abs(ev.real - c) <= dx) and np.all(np.abs(ev.imag) <= dy)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgmres.so not built")
@pytest.mark.parametrize("kind", ["general", "symmetric", "clustered", "defective"])
def test_host_hessenberg_eigenvalues_match_numpy(kind):
    lib = ctypes.CDLL(LIB)
    f = lib.sgmres_hessenberg_eigenvalues
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    rng = np.random.default_rng({"general": 1, "symmetric": 2, "clustered": 3, "defective": 4}[kind])
    worst = 0.0
    for m in list(range(1, 12)) + [20, 33, 64]:
        X = rng.standard_normal((m, m))
        if kind == "symmetric":
            X = X + X.T
        elif kind == "clustered":
            X = np.diag(rng.integers(-3, 4, m).astype(float)) + 1e-3 * X
        elif kind == "defective":  # Jordan-like blocks: eigenvalues 2 (repeated) and -1
            X = np.diag(np.where(np.arange(m) % 2 == 0, 2.0, -1.0)) + np.diag(np.ones(m - 1), 1)
        H = np.triu(X, -1)
        ld = m + 3  # a leading dimension larger than m
        Hc = np.zeros((ld, m), order="F")
        Hc[:m, :] = H
        Hc[m:, :] = 7.0  # below the matrix: must be ignored
        keep = Hc.copy()
        wr, wi = np.zeros(m), np.zeros(m)
        rc = f(m, Hc.ctypes.data, ld, wr.ctypes.data, wi.ctypes.data)
        assert rc == 0
        assert np.array_equal(Hc, keep)  # the input is not modified
        got, ref = wr + 1j * wi, np.linalg.eigvals(H)
        # defective eigenvalues are only accurate to about sqrt(eps)
        tol = 1e-6 if kind == "defective" else 1e-10
        scale = max(1.0, np.abs(ref).max())
        worst = max(worst, nearest_gap(got, ref) / scale, nearest_gap(ref, got) / scale)
        assert worst <= tol, (m, worst)
    print(f"{kind}: worst relative gap {worst:.2e}")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgmres.so not built")
def test_host_hessenberg_eigenvalues_rejects_bad_sizes():
    lib = ctypes.CDLL(LIB)
    f = lib.sgmres_hessenberg_eigenvalues
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    H = np.eye(3, order="F")
    w = np.zeros(3)
    assert f(0, H.ctypes.data, 3, w.ctypes.data, w.ctypes.data) == -1
    assert f(3, H.ctypes.data, 2, w.ctypes.data, w.ctypes.data) == -1
