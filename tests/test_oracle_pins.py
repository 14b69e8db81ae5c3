"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test ties one oracle function to something fixed independently: published
known-answer vectors, a dense or library route (numpy / scipy), a closed form,
an invariant of the method, or a bound the paper proves.  They are chosen so
that a plausible slip (a dropped term, a wrong sign or index, a transposed
operand, a wrong scale, a missing second Gram-Schmidt pass) fails at least one.
"""

import os

import numpy as np
import pytest

import synth

U = 2.0**-53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al., SC'11): published known-answer vectors
# --------------------------------------------------------------------------
def test_philox_known_answers(orc):
    rows = [
        ln.split()
        for ln in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
        if ln.strip() and not ln.startswith("#")
    ]
    assert len(rows) == 3
    for r in rows:
        w = [int(t, 16) for t in r]
        out = orc.philox4x32_10(w[0:4], w[4:6])
        assert list(out) == w[6:10]


# --------------------------------------------------------------------------
# Sparse sign embedding, Section 2.3.2
# --------------------------------------------------------------------------
@pytest.mark.parametrize("s,zeta", [(80, 8), (400, 8), (9, 8), (5, 5), (1, 1), (200, 11)])
def test_pattern_distinct_rows_in_range(orc, s, zeta):
    rows, signs = orc.sketch_pattern(seed=7, cycle=3, i0=1000, count=500, s=s, zeta=zeta)
    assert rows.min() >= 0 and rows.max() < s
    for q in range(rows.shape[0]):
        assert len(set(rows[q].tolist())) == zeta  # exactly zeta nonzeros per column
    assert set(np.unique(signs).tolist()) <= {-1, 1}


def test_pattern_uniform_rows_and_balanced_signs(orc):
    from scipy import stats

    s, zeta, count = 40, 8, 20000
    rows, signs = orc.sketch_pattern(seed=123, cycle=0, i0=0, count=count, s=s, zeta=zeta)
    hist = np.bincount(rows.reshape(-1), minlength=s)
    # each row is hit with probability zeta/s per column
    chi2 = ((hist - count * zeta / s) ** 2 / (count * zeta / s)).sum()
    assert stats.chi2.sf(chi2, s - 1) > 1e-4
    npos = int((signs > 0).sum())
    assert abs(npos - signs.size / 2) < 5 * np.sqrt(signs.size / 4)
    # pairs of rows inside a column are not biased toward neighbours
    gaps = np.abs(rows[:, 1] - rows[:, 0])
    assert 0.25 * s < gaps.mean() < 0.42 * s  # E|X-Y| ~ s/3 for distinct uniform X, Y


def test_pattern_keyed_by_seed_cycle_column(orc):
    a = orc.sketch_pattern(1, 0, 0, 64, 400, 8)[0]
    b = orc.sketch_pattern(1, 0, 0, 64, 400, 8)[0]
    c = orc.sketch_pattern(1, 1, 0, 64, 400, 8)[0]
    d = orc.sketch_pattern(2, 0, 0, 64, 400, 8)[0]
    e = orc.sketch_pattern(1, 0, 1, 64, 400, 8)[0]
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)
    assert np.array_equal(a[1:], e[:-1])  # column i depends on i only, not on the batch
    # high word of the column index enters the counter
    f = orc.sketch_pattern(1, 0, 2**32, 4, 400, 8)[0]
    assert not np.array_equal(a[:4], f)


def _pattern_from_words(orc, seed, cycle, i, s, zeta):
    """The written pattern specification applied to raw Philox4x32-10 blocks:
    key (lo32 seed, hi32 seed), counter (lo32 i, hi32 i, cycle, t); the words
    of blocks t = 0, 1, ... in order, word u proposing row floor(u s / 2^32)
    with sign -1 iff u is odd; repeats of an accepted row skipped."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    rows, signs = [], []
    t = 0
    while len(rows) < zeta:
        words = orc.philox4x32_10([i & 0xFFFFFFFF, i >> 32, cycle, t], key)
        for u in (int(w) for w in words):
            if len(rows) == zeta:
                break
            row = (u * s) >> 32
            if row in rows:
                continue
            rows.append(row)
            signs.append(-1 if u & 1 else 1)
        t += 1
    return rows, signs


@pytest.mark.parametrize("seed,cycle,i0,s,zeta", [(0, 0, 0, 400, 8), (12345678901234, 7, 2**32 - 3, 400, 8),
                                                  (5, 1, 17, 9, 8), (9, 2, 100, 200, 32), (3, 4, 7, 1, 1)])
def test_pattern_follows_written_spec_word_by_word(orc, seed, cycle, i0, s, zeta):
    # Pins the mapping from the Philox words (themselves pinned by the
    # known-answer vectors) to rows and signs: the word order, the row formula
    # and the sign bit.  A sign read from bit 31, or words taken in another
    # order, would pass the statistical pins below but fail here.
    rows, signs = orc.sketch_pattern(seed, cycle, i0, 6, s, zeta)
    for q in range(6):
        r_ref, s_ref = _pattern_from_words(orc, seed, cycle, i0 + q, s, zeta)
        assert rows[q].tolist() == r_ref
        assert signs[q].tolist() == s_ref


def test_pattern_sign_independent_of_row(orc):
    # the sign bit (bit 0 of the word) is independent of the row, which the top
    # bits decide: in the upper and the lower half of the rows about half the
    # signs are negative (a sign taken from bit 31 would make every upper-half
    # row negative)
    rows, signs = orc.sketch_pattern(seed=77, cycle=1, i0=0, count=5000, s=400, zeta=8)
    for half in (rows < 200, rows >= 200):
        neg = float((signs[half] < 0).mean())
        assert abs(neg - 0.5) < 0.02


def test_oracle_bits_independent_of_thread_count(orc):
    # every sum over rows runs in fixed chunks of 4096 rows, so threads only
    # spread the work: a cycle and a restarted solve give identical bits
    A = synth.convection_diffusion(100, (50.0, 20.0))  # n = 10,000: three chunks, ragged tail
    f = synth.rhs(A.n, 0)
    outs = []
    try:
        for t in (1, 3, 8):
            orc.set_threads(t)
            c = orc.arnoldi_cycle(A, f, 20, 4, 40, 8, 5, 1)
            rc, x, info = orc.sgmres_solve(A, f, d=20, k=4, s=40, seed=5, tol=1e-12, restarts=4)
            outs.append((c, x, info))
    finally:
        orc.set_threads(1)
    for c, x, info in outs[1:]:
        for key in ("B", "SB", "SAB", "H", "g"):
            assert np.array_equal(c[key], outs[0][0][key]), key
        assert np.array_equal(x, outs[0][1])
        assert info == outs[0][2]


def test_sketch_apply_matches_dense_matrix(orc):
    rng = np.random.default_rng(0)
    n, s, zeta = 300, 50, 8
    S = orc.sketch_dense(n, seed=5, cycle=2, s=s, zeta=zeta)
    assert np.allclose((S != 0).sum(axis=0), zeta)
    assert np.allclose(np.abs(S[S != 0]), 1 / np.sqrt(zeta))
    for _ in range(3):
        v = rng.standard_normal(n)
        g = orc.sketch_apply(v, seed=5, cycle=2, s=s, zeta=zeta)
        assert np.allclose(g, S @ v, rtol=1e-14, atol=1e-14 * np.abs(v).sum())


def test_sketch_is_isometric_in_expectation(orc):
    # E|Sx|^2 = |x|^2 for columns with zeta distinct rows, independent signs and
    # scale 1/sqrt(zeta).  A 1/sqrt(s) scale would give zeta/s = 0.1 here.
    rng = np.random.default_rng(1)
    n, s, zeta = 400, 80, 8
    x = rng.standard_normal(n)
    ratios = [np.sum(orc.sketch_apply(x, seed=sd, cycle=0, s=s, zeta=zeta) ** 2) / np.sum(x**2)
              for sd in range(300)]
    assert abs(np.mean(ratios) - 1.0) < 0.03


def test_embedding_distortion_near_paper_value(orc):
    # Section 3.3: s = 2(d+1) typically gives distortion about 1/sqrt(2); the
    # embedding definition (Section 2) is checked on the singular values of SQ.
    rng = np.random.default_rng(2)
    n, d1 = 2000, 21
    s = 2 * d1
    Q, _ = np.linalg.qr(rng.standard_normal((n, d1)))
    eps = []
    for seed in range(40):
        S = orc.sketch_dense(n, seed=seed, cycle=0, s=s, zeta=8)
        sv = np.linalg.svd(S @ Q, compute_uv=False)
        eps.append(max(sv[0] - 1, 1 - sv[-1]))
    eps = np.array(eps)
    assert np.mean(eps < 0.8) >= 0.95
    assert 0.5 < np.median(eps) < 0.8  # Marchenko-Pastur edge 1 - sqrt(d1/s) = 0.29 -> eps ~ 0.71


# --------------------------------------------------------------------------
# Matrix access and the operator generators
# --------------------------------------------------------------------------
def test_spmv_exact_on_integers(orc):
    rng = np.random.default_rng(3)
    n = 64
    A = synth.random_dominant(n, offdiag=6, seed=9)
    A.val = np.round(A.val * 8)  # integer values keep every sum exact
    x = rng.integers(-50, 50, n).astype(np.float64)
    assert np.array_equal(orc.csr_spmv(A, x), A.to_dense() @ x)


def test_residual_definition(orc):
    rng = np.random.default_rng(4)
    A = synth.convection_diffusion(9, (3.0, -2.0))
    f, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    r, nrm = orc.residual(A, f, x)
    ref = f - A.to_dense() @ x
    assert np.allclose(r, ref, rtol=1e-14, atol=1e-14)
    assert np.isclose(nrm, np.linalg.norm(ref), rtol=1e-14)


def test_csr_transpose_matches_dense(orc):
    A = synth.random_dominant(200, offdiag=6, seed=11)
    At = orc.csr_transpose(A)
    assert np.array_equal(At.to_dense(), A.to_dense().T)
    for i in range(At.n):  # columns sorted inside each row
        seg = At.col_idx[At.row_ptr[i]:At.row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_convection_diffusion_matches_kronecker_form():
    import scipy.sparse as sp

    N, bx, by = 12, 50.0, 20.0
    h = 1.0 / (N + 1)
    A = synth.convection_diffusion(N, (bx, by))
    assert A.nnz == 5 * N * N - 4 * N
    I = sp.identity(N)
    second = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(N, N))
    first = sp.diags([-1, 1], [-1, 1], shape=(N, N)) * (h / 2)
    ref = sp.kron(I, second) + sp.kron(second, I) + bx * sp.kron(I, first) + by * sp.kron(first, I)
    assert np.allclose(A.to_dense(), ref.toarray(), rtol=0, atol=1e-15)


def test_random_dominant_rows():
    A = synth.random_dominant(500, offdiag=6, seed=[4, 3])
    D = A.to_dense()
    off = np.abs(D).sum(axis=1) - np.abs(np.diag(D))
    assert np.allclose(np.diag(D), 1.2 * off)
    assert np.all(np.diff(A.row_ptr) == 7)


# --------------------------------------------------------------------------
# k-truncated Arnoldi with double Gram-Schmidt (Section 1.2.2, Algorithm 1)
# --------------------------------------------------------------------------
def _cycle(orc, A, d, k, s=None, seed=0, passes=2, r=None):
    r = synth.rhs(A.n, 5) if r is None else r
    s = 2 * d if s is None else s
    return r, orc.arnoldi_cycle(A, r, d, k, s, 8, seed, 0, passes)


def test_basis_columns_unit_and_locally_orthogonal(orc):
    A = synth.convection_diffusion(20, (50.0, 20.0))
    d, k = 30, 4
    _, c = _cycle(orc, A, d, k)
    B = c["B"]
    G = B.T @ B
    assert np.allclose(np.diag(G), 1.0, atol=20 * U)
    for i in range(d):
        for j in range(max(0, i - k), i):
            assert abs(G[i, j]) < 200 * U, (i, j, G[i, j])
    # columns further apart than k are not orthogonalised and are visibly not orthogonal
    far = max(abs(G[i, j]) for i in range(d) for j in range(0, i - k - 1))
    assert far > 1e-6


def test_arnoldi_relation(orc):
    # A b_j = sum_{a<kw} H[a,j] b_{j-a} + nu_j b_{j+1}  (banded Hessenberg form)
    A = synth.random_dominant(300, offdiag=6, seed=21)
    Ad = A.to_dense()
    d, k = 25, 3
    r, c = _cycle(orc, A, d, k)
    B, H = c["B"], c["H"]
    for j in range(d - 1):
        kw = min(j + 1, k)
        rhs = sum(H[a, j] * B[:, j - a] for a in range(kw)) + H[k, j] * B[:, j + 1]
        assert np.linalg.norm(Ad @ B[:, j] - rhs) < 100 * U * np.linalg.norm(Ad, 2)
    assert np.allclose(B[:, 0], r / np.linalg.norm(r), rtol=0, atol=4 * U)


def test_basis_spans_krylov_space(orc):
    A = synth.random_dominant(200, offdiag=6, seed=22)
    Ad = A.to_dense()
    d, k = 6, 2
    r, c = _cycle(orc, A, d, k)
    K = np.empty((A.n, d))
    v = r / np.linalg.norm(r)
    for j in range(d):
        K[:, j] = v
        v = Ad @ v
        v /= np.linalg.norm(v)
    Qb, _ = np.linalg.qr(c["B"])
    resid = K - Qb @ (Qb.T @ K)
    assert np.linalg.norm(resid) < 1e-10
    # and the sketches are S applied to the basis and to the reduced matrix
    S = orc.sketch_dense(A.n, 0, 0, 2 * d, 8)
    assert np.allclose(c["SB"], S @ c["B"], rtol=1e-13, atol=1e-13)
    assert np.allclose(c["SAB"], S @ (Ad @ c["B"]), rtol=1e-12, atol=1e-12)
    assert np.allclose(c["g"], S @ r, rtol=1e-13, atol=1e-13)


def test_full_orthogonalisation_is_orthonormal(orc):
    # k >= d-1 reduces truncated Arnoldi to the Arnoldi process (Section 4.2)
    A = synth.convection_diffusion(15, (50.0, 20.0))
    d = 40
    _, c = _cycle(orc, A, d, d - 1)
    B = c["B"]
    assert np.linalg.norm(B.T @ B - np.eye(d)) < 1e-13


def test_second_gram_schmidt_pass_restores_orthogonality(orc):
    # A = I + 1e-7 R: A b ~ b, so the first pass cancels almost everything and
    # leaves O(u / 1e-7) components along the window; the second pass removes them.
    base = synth.random_dominant(400, offdiag=6, seed=23)
    R = base.to_dense() / np.abs(base.val).max()
    Ad = np.eye(400) + 1e-7 * R
    rows, cols = np.nonzero(Ad)
    A = synth.problems._csr_from_coo(400, rows, cols, Ad[rows, cols])
    d, k = 12, 2
    _, c2 = _cycle(orc, A, d, k, passes=2)
    _, c1 = _cycle(orc, A, d, k, passes=1)

    def loss(B):
        return max(abs(B[:, i] @ B[:, i - 1]) for i in range(1, d))

    assert loss(c2["B"]) < 100 * U
    assert loss(c1["B"]) > 1e4 * loss(c2["B"])


# --------------------------------------------------------------------------
# Sketched least squares (Section 3.3) and the kappa guard (Sections 3.4, 5.3)
# --------------------------------------------------------------------------
def test_lsq_matches_lstsq_and_qr(orc):
    rng = np.random.default_rng(6)
    s, d = 60, 25
    C = rng.standard_normal((s, d)) @ np.diag(np.logspace(0, -6, d))
    g = rng.standard_normal(s)
    out = orc.sketched_lsq(C, g)
    assert out["d_eff"] == d and out["flags"] == 0
    y_ref = np.linalg.lstsq(C, g, rcond=None)[0]
    assert np.allclose(out["y"], y_ref, rtol=1e-9, atol=0)
    assert np.isclose(out["rest"], np.linalg.norm(C @ out["y"] - g), rtol=1e-10)
    R = np.linalg.qr(C, mode="r")
    assert np.allclose(np.abs(out["T"]), np.abs(R), rtol=1e-10, atol=1e-13)
    # Q^T g keeps the norm of g
    assert np.isclose(np.linalg.norm(out["QTg"]), np.linalg.norm(g), rtol=1e-14)
    # the diagonal ratio bounds the 2-norm condition number from below
    kap2 = np.linalg.cond(out["T"])
    assert out["kappa"] <= kap2 * (1 + 1e-12)


def test_lsq_householder_sign_convention(orc):
    # beta = -sign(alpha)|x|: a column with positive leading entry gets T_11 < 0.
    C = np.array([[3.0, 1.0], [4.0, 2.0], [0.0, 1.0]])
    out = orc.sketched_lsq(C, np.array([1.0, 0.0, 0.0]))
    assert np.isclose(out["T"][0, 0], -5.0)
    C2 = np.array([[-3.0, 1.0], [4.0, 2.0], [0.0, 1.0]])
    assert np.isclose(orc.sketched_lsq(C2, np.ones(3))["T"][0, 0], 5.0)


def test_lsq_kappa_prefix_truncation(orc):
    rng = np.random.default_rng(7)
    s, d = 40, 12
    C = rng.standard_normal((s, d))
    C[:, 8] = C[:, 0:8] @ rng.standard_normal(8) + 1e-13 * rng.standard_normal(s)
    g = rng.standard_normal(s)
    out = orc.sketched_lsq(C, g, kappa_max=1e8)
    assert out["d_eff"] == 8
    assert out["flags"] & orc.FLAG_KAPPA_TRUNC
    y_ref = np.linalg.lstsq(C[:, :8], g, rcond=None)[0]
    assert np.allclose(out["y"], y_ref, rtol=1e-10)
    assert np.isclose(out["rest"], np.linalg.norm(C[:, :8] @ y_ref - g), rtol=1e-10)


def test_basis_combine(orc):
    rng = np.random.default_rng(8)
    B = rng.standard_normal((50, 7))
    y = rng.standard_normal(5)
    x = rng.standard_normal(50)
    assert np.allclose(orc.basis_combine(B, y, x), x + B[:, :5] @ y, rtol=1e-14, atol=1e-14)


# --------------------------------------------------------------------------
# sGMRES as a whole (Sections 3.2-3.5)
# --------------------------------------------------------------------------
def test_sgmres_a_priori_and_a_posteriori_bounds(orc):
    # eq. sgmres-residual: |A x_hat - f| <= (smax/smin)(S Q) |A x_B - f|, where
    # x_B minimises over the same basis without sketching and Q spans [AB, r0];
    # eq. sgmres-residual-norm: r_est in [smin, smax](SQ) * |A x_hat - f|.
    A = synth.convection_diffusion(16, (50.0, 20.0))
    Ad = A.to_dense()
    f = synth.rhs(A.n, 0)
    d, k, s = 20, 2, 42
    for seed in range(5):
        rc, x, info = orc.sgmres_solve(A, f, d=d, k=k, s=s, seed=seed, tol=0.0, restarts=0)
        assert rc == orc.NOT_CONVERGED and info["cycles"] == 1
        c = orc.arnoldi_cycle(A, f, d, k, s, 8, seed, 0)
        AB = Ad @ c["B"]
        yB = np.linalg.lstsq(AB, f, rcond=None)[0]
        resB = np.linalg.norm(AB @ yB - f)
        res_hat = np.linalg.norm(Ad @ x - f)
        Q, _ = np.linalg.qr(np.column_stack([AB, f]))
        S = orc.sketch_dense(A.n, seed, 0, s, 8)
        sv = np.linalg.svd(S @ Q, compute_uv=False)
        assert resB * (1 - 1e-10) <= res_hat <= sv[0] / sv[-1] * resB * (1 + 1e-8)
        rest = info["rest_est"] * np.linalg.norm(f)
        assert sv[-1] * res_hat * (1 - 1e-8) <= rest <= sv[0] * res_hat * (1 + 1e-8)
        assert np.isclose(info["relres"], res_hat / np.linalg.norm(f), rtol=1e-12)


def test_exact_solution_when_basis_is_whole_space(orc):
    # d = n: the Krylov space is the whole space (Section 4.1), so x_hat = A^{-1} f
    A = synth.random_dominant(30, offdiag=4, seed=31)
    Ad = A.to_dense()
    f = synth.rhs(30, 1)
    x_ref = np.linalg.solve(Ad, f)
    for k in (29, 2):
        rc, x, info = orc.sgmres_solve(A, f, d=30, k=k, s=62, tol=0.0, restarts=0)
        assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e3 * np.linalg.cond(Ad) * U


def test_lucky_breakdown_gives_exact_solution(orc):
    n = 50
    A = synth.diagonal(np.arange(1.0, n + 1))
    f = np.zeros(n)
    f[0] = f[1] = 1.0
    c = orc.arnoldi_cycle(A, f, 10, 2, 22, 8, 0, 0)
    assert c["dc"] == 2 and c["flags"] & orc.FLAG_BREAKDOWN
    rc, x, info = orc.sgmres_solve(A, f, d=10, k=2, s=22, tol=1e-14, restarts=3)
    assert rc == orc.OK and info["cycles"] == 1 and info["steps"] == 2
    assert np.allclose(x[:2], [1.0, 0.5], rtol=1e-14) and np.all(x[2:] == 0)


def test_restarted_solve_reaches_tolerance(orc):
    A, f, p = synth.workload("cd64")
    rc, x, info = orc.sgmres_solve(A, f, d=p["d"], k=p["k"], s=p["s"], seed=0, tol=1e-10, restarts=50)
    assert rc == orc.OK
    true = np.linalg.norm(f - A.to_scipy() @ x) / np.linalg.norm(f)
    assert true <= 1e-10 and np.isclose(true, info["relres"], rtol=1e-8)
    assert info["steps"] == info["cycles"] * p["d"]


def test_transposed_solve(orc):
    A = synth.convection_diffusion(16, (50.0, 20.0))
    f = synth.rhs(A.n, 2)
    rc, x, info = orc.sgmres_solve_transposed(A, f, d=40, k=2, s=80, tol=1e-10, restarts=50)
    assert rc == orc.OK
    assert np.linalg.norm(f - A.to_dense().T @ x) / np.linalg.norm(f) <= 1e-10


def test_zero_rhs_and_argument_errors(orc):
    A = synth.convection_diffusion(8)
    rc, x, info = orc.sgmres_solve(A, np.zeros(A.n), x0=np.ones(A.n), d=10, k=2, s=22)
    assert rc == orc.OK and np.all(x == 0) and info["relres"] == 0
    f = synth.rhs(A.n)
    assert orc.sgmres_solve(A, f, d=10, k=2, s=10)[0] == -1  # s < d + 1
    assert orc.sgmres_solve(A, f, d=A.n + 1, k=2, s=2 * A.n + 4)[0] == -1  # d > n
    assert orc.sgmres_solve(A, f, d=10, k=0, s=22)[0] == -1
    assert orc.sgmres_solve(A, f, d=10, k=2, s=22, zeta=23)[0] == -1
    bad = f.copy()
    bad[3] = np.nan
    assert orc.sgmres_solve(A, bad, d=10, k=2, s=22)[0] == -5


# --------------------------------------------------------------------------
# Adjoint gradient of a solve (dense FP64 reference for the differentiable solve)
# --------------------------------------------------------------------------
def test_dense_gradient_matches_finite_differences(orc):
    A = synth.random_dominant(30, offdiag=4, seed=41)
    rng = np.random.default_rng(5)
    b, xt = rng.standard_normal(30), rng.standard_normal(30)
    x, L, gb, gval = orc.dense_solve_gradient(A, b, xt)

    def loss(val, bb):
        B = synth.CSR(A.n, A.row_ptr, A.col_idx, val)
        return orc.dense_solve_gradient(B, bb, xt)[1]

    h = 1e-6
    for q in rng.choice(A.nnz, 12, replace=False):
        vp, vm = A.val.copy(), A.val.copy()
        vp[q] += h
        vm[q] -= h
        fd = (loss(vp, b) - loss(vm, b)) / (2 * h)
        assert abs(fd - gval[q]) <= 1e-6 * max(1.0, abs(gval[q]))
    for i in rng.choice(30, 6, replace=False):
        bp, bm = b.copy(), b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss(A.val, bp) - loss(A.val, bm)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-6 * max(1.0, abs(gb[i]))


# --------------------------------------------------------------------------
# Chebyshev basis, Section 4.4.  On a diagonal matrix the recurrence acts
# entrywise, so column j (0-based) is b_1 times a degree-j polynomial of the
# eigenvalue.  For a box [c +- dx] x [+-dy] with dx != dy it is
# sigma^j T_j((lambda - c)/f) with f = sqrt(dx^2 - dy^2) (imaginary when
# dy > dx; the powers of i then cancel) and sigma = f / (2 rho),
# rho = max(dx, dy).  numpy's Chebyshev evaluator is the independent route.
# --------------------------------------------------------------------------
def _cheb_columns(lam, b1, d, c, dx, dy):
    from numpy.polynomial import chebyshev as C

    rho = max(dx, dy)
    f = np.sqrt(complex(dx * dx - dy * dy))
    sigma = f / (2 * rho)
    cols, raw = [], []
    for j in range(d):
        v = b1 * C.chebval((lam - c) / f, [0] * j + [1]) * sigma**j
        assert np.abs(v.imag).max() <= 1e-12 * np.abs(v.real).max()
        v = v.real
        raw.append(np.linalg.norm(v))
        cols.append(v / np.linalg.norm(v))
    return np.array(cols).T, np.array(raw)


@pytest.mark.parametrize("c,dx,dy", [(4.0, 4.0, 0.0), (4.0, 4.0, 2.5), (3.0, 2.0, 3.5)])
def test_chebyshev_basis_closed_form_on_diagonal(orc, c, dx, dy):
    n, d = 64, 12
    lam = np.linspace(c - dx, c + dx, n)
    A = synth.diagonal(lam)
    r = np.random.default_rng(7).standard_normal(n)
    out = orc.chebyshev_cycle(A, r, d, 30, 4, 3, 1, c, dx, dy)
    ref, raw = _cheb_columns(lam, r / np.linalg.norm(r), d, c, dx, dy)
    assert np.abs(out["B"] - ref).max() <= 1e-12
    # the paper's unnormalised scaling: |b_j| = |sigma|^j |T_j(u) b_1|
    np.testing.assert_allclose(out["nrm"], raw, rtol=1e-12)


def test_chebyshev_disk_box_gives_monomials(orc):
    # dx = dy: gamma = 0, the recurrence is b_{j+1} = (A - c) b_j / rho (halved once)
    n, d, c, rho = 40, 8, 2.0, 1.5
    lam = np.linspace(0.7, 3.3, n)
    A = synth.diagonal(lam)
    r = np.random.default_rng(8).standard_normal(n)
    out = orc.chebyshev_cycle(A, r, d, 20, 4, 0, 0, c, rho, rho)
    b1 = r / np.linalg.norm(r)
    for j in range(d):
        v = b1 * ((lam - c) / rho) ** j * (0.5 if j >= 1 else 1.0)
        assert np.abs(out["B"][:, j] - v / np.linalg.norm(v)).max() <= 1e-13
        assert abs(out["nrm"][j] - np.linalg.norm(v)) <= 1e-13 * np.linalg.norm(v)


def test_chebyshev_sketches_match_dense_sketch(orc):
    A = synth.convection_diffusion(12, (10.0, 10.0))
    r = np.random.default_rng(9).standard_normal(A.n)
    d, s, zeta, seed, cyc = 10, 30, 5, 11, 2
    out = orc.chebyshev_cycle(A, r, d, s, zeta, seed, cyc, 4.0, 4.0, 0.0)
    S = orc.sketch_dense(A.n, seed, cyc, s, zeta)
    D = A.to_dense()
    np.testing.assert_allclose(out["SB"], S @ out["B"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(out["SAB"], S @ (D @ out["B"]), rtol=0, atol=1e-13)
    np.testing.assert_allclose(out["g"], S @ r, rtol=0, atol=1e-13)
    # columns have unit norm and span the Krylov space K_d(A, r)
    np.testing.assert_allclose(np.linalg.norm(out["B"], axis=0), 1.0, rtol=1e-14)
    K = np.empty((A.n, d))
    K[:, 0] = r / np.linalg.norm(r)
    for j in range(1, d):
        K[:, j] = D @ K[:, j - 1]
        K[:, j] /= np.linalg.norm(K[:, j])
    Q, _ = np.linalg.qr(K)
    assert np.linalg.norm(out["B"] - Q @ (Q.T @ out["B"])) <= 1e-9


def test_chebyshev_solve_exact_on_whole_space(orc):
    # d = n: the basis spans R^n, so one cycle solves the system (Section 3)
    A = synth.random_dominant(16, offdiag=4, seed=3)
    ev = np.linalg.eigvals(A.to_dense())
    c = 0.5 * (ev.real.max() + ev.real.min())
    dx = 0.5 * (ev.real.max() - ev.real.min()) * 1.05
    dy = np.abs(ev.imag).max() * 1.05
    b = np.random.default_rng(4).standard_normal(16)
    rc, x, info = orc.sgmres_solve_chebyshev(A, b, (c, dx, dy), d=16, s=40, zeta=6, tol=0.0, restarts=0)
    x_ref = np.linalg.solve(A.to_dense(), b)
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


def test_chebyshev_restarted_solve_reaches_tolerance(orc):
    A = synth.convection_diffusion(24, (10.0, 10.0))
    b = synth.rhs(A.n, 0)
    rc, x, info = orc.sgmres_solve_chebyshev(A, b, (4.0, 4.0, 0.0), d=40, s=90, zeta=8, tol=1e-10, restarts=200)
    assert rc == orc.OK
    assert info["relres"] <= 1e-10
    r = b - A.to_scipy() @ x
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)


def test_chebyshev_rejects_empty_box(orc):
    A = synth.diagonal(np.ones(5))
    with pytest.raises(ValueError):
        orc.chebyshev_cycle(A, np.ones(5), 2, 4, 2, 0, 0, 1.0, 0.0, 0.0)
