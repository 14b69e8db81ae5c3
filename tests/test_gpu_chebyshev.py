"""GPU parity of the Chebyshev basis (Section 4.4) against the CPU oracle.

The GPU keeps the raw recurrence vectors rescaled by a constant kappa per
step (kappa = 2 rho / (dx + dy)) and reports their norms; the oracle runs the
recurrence in the paper's scaling.  Compared: the normalised columns, S B and
S A B of the normalised columns, g = S r, and colnorm against kappa^j times the
oracle's norms.  Tolerances as for the Arnoldi basis: one-pass sketches to
~1e-12 of the column scale, the recurrence (no reorthogonalisation) to 1e-10
on unit columns over the short cycles here, one-cycle solutions to 1e-9.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def sg():
    import paper_2111_00113_amd as sg

    sg.lib()
    return sg


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _gershgorin_box(A):
    """Box [c +- dx] x [+-dy] containing every Gershgorin disc of A."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    diag = np.zeros(A.n)
    rad = np.zeros(A.n)
    on = rows == A.col_idx
    np.add.at(diag, rows[on], A.val[on])
    np.add.at(rad, rows[~on], np.abs(A.val[~on]))
    lo, hi = (diag - rad).min(), (diag + rad).max()
    return 0.5 * (lo + hi), 0.5 * (hi - lo), rad.max()


def _kappa(dx, dy):
    return 2.0 * max(dx, dy) / (dx + dy)


def _compare_cycle(out, ref, d, dx, dy, col_tol=1e-10):
    cn = _np(out["colnorm"])
    B = _np(out["B"]) / np.where(cn > 0, cn, 1.0)
    Bref = ref["B"]
    for j in range(d):
        assert np.linalg.norm(B[:, j] - Bref[:, j]) <= col_tol, j
    np.testing.assert_allclose(cn, _kappa(dx, dy) ** np.arange(d) * ref["nrm"], rtol=1e-10)
    for key in ("SB", "SAB"):
        M, Mref = _np(out[key]), ref[key]
        scale = np.abs(Mref).max(axis=0) + 1e-300
        assert np.all(np.abs(M - Mref).max(axis=0) <= 1e-10 * scale), key
    g = _np(out["g"])
    assert np.abs(g - ref["g"]).max() <= 1e-12 * np.abs(ref["g"]).max()


@pytest.mark.parametrize(
    "case",
    [
        "cd100_interval",  # n = 10,000: several workgroups and a ragged tail
        "cd64_ellipse",
        "rand_gershgorin",  # nonsymmetric, box with dy > 0 from Gershgorin discs
        "cd30_tall",  # imaginary foci (dy > dx)
    ],
)
def test_chebyshev_cycle_parity(sg, orc, case):
    if case == "cd100_interval":
        A = synth.convection_diffusion(100, (30.0, 10.0))
        box, d, s, zeta = (4.0, 4.0, 0.0), 30, 70, 8
    elif case == "cd64_ellipse":
        A = synth.convection_diffusion(64, (10.0, 10.0))
        box, d, s, zeta = (4.0, 4.2, 1.0), 24, 60, 6
    elif case == "rand_gershgorin":
        A = synth.random_dominant(7001, offdiag=6, seed=5)
        box, d, s, zeta = _gershgorin_box(A), 16, 40, 8
    else:
        A = synth.convection_diffusion(30)
        box, d, s, zeta = (4.0, 3.0, 4.5), 12, 30, 4
    r = synth.rhs(A.n, 2)
    c, dx, dy = box
    out = sg.sgmres_chebyshev_cycle(sg.DeviceCSR.from_host(A), _t(r), d, s, c, dx, dy, zeta, 17, 3)
    ref = orc.chebyshev_cycle(A, r, d, s, zeta, 17, 3, c, dx, dy)
    _compare_cycle(out, ref, d, dx, dy)


def test_chebyshev_cycle_d1_and_zero_column(sg, orc):
    # d = 1: no recurrence step.  A = 2 I with c = 2: (A - cI) b_1 = 0, so column 2
    # has norm 0 and zero sketches on both sides; column 3 restarts from b_1.
    A = synth.diagonal(np.full(3000, 2.0))
    r = synth.rhs(A.n, 1)
    dA = sg.DeviceCSR.from_host(A)
    out = sg.sgmres_chebyshev_cycle(dA, _t(r), 1, 8, 2.0, 1.0, 0.0, 4, 0, 0)
    ref = orc.chebyshev_cycle(A, r, 1, 8, 4, 0, 0, 2.0, 1.0, 0.0)
    _compare_cycle(out, ref, 1, 1.0, 0.0)
    out = sg.sgmres_chebyshev_cycle(dA, _t(r), 3, 8, 2.0, 1.0, 0.0, 4, 0, 0)
    ref = orc.chebyshev_cycle(A, r, 3, 8, 4, 0, 0, 2.0, 1.0, 0.0)
    assert float(out["colnorm"][1]) == 0.0 and ref["nrm"][1] == 0.0
    assert float(out["SAB"][:, 1].abs().max()) == 0.0 and float(out["SB"][:, 1].abs().max()) == 0.0
    _compare_cycle(out, ref, 3, 1.0, 0.0)


def test_chebyshev_one_cycle_solution(sg, orc):
    A = synth.convection_diffusion(80, (20.0, 20.0))
    f = synth.rhs(A.n, 4)
    dA = sg.DeviceCSR.from_host(A)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    rc, info = sg.sgmres_solve(dA, _t(f), x, 40, 1, 90, 5, 0.0, 0, cheb_box=(4.0, 4.0, 0.0))
    rc_o, x_o, info_o = orc.sgmres_solve_chebyshev(A, f, (4.0, 4.0, 0.0), d=40, s=90, zeta=8, seed=5, tol=0.0,
                                                   restarts=0)
    xg = _np(x)
    assert info["cycles"] == 1 and info_o["cycles"] == 1
    assert info["d_eff_last"] == info_o["d_eff_last"]
    assert np.linalg.norm(xg - x_o) <= 1e-9 * np.linalg.norm(x_o)
    assert abs(info["relres"] - info_o["relres"]) <= 1e-10


def test_chebyshev_restarted_solve(sg, orc):
    A = synth.convection_diffusion(96, (50.0, 20.0))
    f = synth.rhs(A.n, 0)
    dA = sg.DeviceCSR.from_host(A)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    rc, info = sg.sgmres_solve(dA, _t(f), x, 60, 1, 130, 0, 1e-10, 500, cheb_box=(4.0, 4.0, 0.0))
    rc_o, x_o, info_o = orc.sgmres_solve_chebyshev(A, f, (4.0, 4.0, 0.0), d=60, s=130, zeta=8, seed=0, tol=1e-10,
                                                   restarts=500)
    assert rc == sg.OK and rc_o == orc.OK
    _, nrm = orc.residual(A, f, _np(x))
    assert nrm / np.linalg.norm(f) <= 1e-10
    # the same restarted iteration: cycle counts agree up to rounding drift
    assert abs(info["cycles"] - info_o["cycles"]) <= max(1, info_o["cycles"] // 10)


def test_chebyshev_barrier_modes_bit_identical(sg, orc):
    A = synth.convection_diffusion(256, (50.0, 20.0))
    f = _t(synth.rhs(A.n, 0))
    dA = sg.DeviceCSR.from_host(A)
    outs = []
    for mode in (0, 1, 0):
        x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
        rc, info = sg.sgmres_solve(dA, f, x, 60, 1, 120, 3, 0.0, 2, barrier_mode=mode, cheb_box=(4.0, 4.0, 0.0))
        outs.append((_np(x), info["relres"]))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0])
        assert o[1] == outs[0][1]


def test_chebyshev_rejects_bad_box(sg):
    A = synth.convection_diffusion(10)
    dA = sg.DeviceCSR.from_host(A)
    f = _t(synth.rhs(A.n))
    # (dx, dy) = (0, 0) asks the solve to estimate the box (see below); the
    # cycle entry point, which takes the box as given, rejects it
    for box in [(4.0, 0.0, 0.0), (4.0, -1.0, 0.0), (float("nan"), 1.0, 0.0), (4.0, float("inf"), 0.0)]:
        if box[1] != 0.0:
            x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
            with pytest.raises(sg.SGMRESError) as e:
                sg.sgmres_solve(dA, f, x, 10, 1, 22, cheb_box=box)
            assert e.value.rc == -1
        with pytest.raises(sg.SGMRESError):
            sg.sgmres_chebyshev_cycle(dA, f, 4, 10, *box)


# ---------------------------------------------------------------- box estimate
def _nearest_gap(a, b):
    return max(min(abs(x - y) for x in a) for y in b)


def test_box_estimate_matches_oracle(sg, orc):
    """m + 1 Arnoldi steps on the GPU (full window, two Gram-Schmidt passes)
    against the oracle's: the same Ritz values to rounding, the same box."""
    for N, beta, m in [(64, (10.0, 10.0), 20), (50, (50.0, 20.0), 12), (40, (0.0, 0.0), 30)]:
        A = synth.convection_diffusion(N, beta)
        f = synth.rhs(A.n, 2)
        box, ritz = sg.sgmres_chebyshev_box(sg.DeviceCSR.from_host(A), _t(f), m)
        th = orc.ritz_values(A, f, m)
        box_o = orc.chebyshev_box(A, f, m)
        scale = np.abs(th).max()
        print(f"cd{N} beta={beta} m={m}: box {box}, oracle {box_o}", flush=True)
        assert len(ritz) == len(th) == m
        assert _nearest_gap(ritz, th) <= 1e-8 * scale and _nearest_gap(th, ritz) <= 1e-8 * scale
        assert np.allclose(box, box_o, rtol=1e-8, atol=1e-10 * scale)


def test_box_estimate_invariant_subspace(sg):
    # A = diag(A1, A2), r supported on A1's rows: the basis stops after q
    # columns and the Ritz values are eig(A1) (numpy on the dense block)
    import scipy.sparse as sps

    rng = np.random.default_rng(3)
    q, n = 7, 40
    A1 = rng.standard_normal((q, q)) + 3.0 * np.eye(q)
    Ad = np.zeros((n, n))
    Ad[:q, :q] = A1
    Ad[q:, q:] = rng.standard_normal((n - q, n - q))
    M = sps.csr_matrix(Ad)
    A = synth.CSR(n=n, row_ptr=M.indptr.astype(np.int32), col_idx=M.indices.astype(np.int32),
                  val=M.data.astype(np.float64))
    r = np.zeros(n)
    r[:q] = rng.standard_normal(q)
    box, ritz = sg.sgmres_chebyshev_box(sg.DeviceCSR.from_host(A), _t(r), 12)
    ev = np.linalg.eigvals(A1)
    assert len(ritz) == q
    assert _nearest_gap(ritz, ev) <= 1e-10 * np.abs(ev).max()
    assert np.all(np.abs(ev.real - box[0]) <= box[1]) and np.all(np.abs(ev.imag) <= box[2])


def test_box_estimate_edge_cases(sg):
    A = synth.convection_diffusion(12)
    dA = sg.DeviceCSR.from_host(A)
    z = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    box, ritz = sg.sgmres_chebyshev_box(dA, z, 5)  # r = 0: a valid box, no Ritz values
    assert box == (0.0, 1.0, 0.0) and len(ritz) == 0
    f = _t(synth.rhs(A.n, 1))
    for m in (0, 65, A.n):
        with pytest.raises(sg.SGMRESError):
            sg.sgmres_chebyshev_box(dA, f, m)
    bad = f.clone()
    bad[3] = float("nan")
    with pytest.raises(sg.SGMRESError):
        sg.sgmres_chebyshev_box(dA, bad, 5)


def test_chebyshev_solve_with_estimated_box(sg, orc):
    """cheb_box="auto": the solve estimates the box from b with
    m = min(20, d, n - 1) (the same box sgmres_chebyshev_box returns, bit for
    bit), and converges like the oracle's Chebyshev solve with the oracle's
    estimate of the box."""
    A = synth.convection_diffusion(96, (50.0, 20.0))
    f = synth.rhs(A.n, 0)
    dA = sg.DeviceCSR.from_host(A)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    rc, info = sg.sgmres_solve(dA, _t(f), x, 60, 1, 130, 0, 1e-10, 500, cheb_box="auto")
    box, _ = sg.sgmres_chebyshev_box(dA, _t(f), 20)
    assert info["path"] == sg.PATH_CHEBYSHEV and tuple(info["cheb_box"]) == box
    box_o = orc.chebyshev_box(A, f, 20)
    rc_o, x_o, info_o = orc.sgmres_solve_chebyshev(A, f, box_o, d=60, s=130, zeta=8, seed=0, tol=1e-10,
                                                   restarts=500)
    _, nrm = orc.residual(A, f, _np(x))
    print(f"estimated box {box} (oracle {box_o}); cycles {info['cycles']} (oracle {info_o['cycles']}, "
          f"given box (4, 4, 0): see test_chebyshev_restarted_solve)", flush=True)
    assert rc == sg.OK and rc_o == orc.OK
    assert nrm / np.linalg.norm(f) <= 1e-10
    assert abs(info["cycles"] - info_o["cycles"]) <= max(1, info_o["cycles"] // 10)


def test_chebyshev_full_size_first_steps_parity(sg, orc):
    """n = 2^20 operator and launch shape of the benchmark (s = 400, zeta = 8);
    first 12 Chebyshev columns against the oracle."""
    A, f, p = synth.workload("cd1024")
    d = 12
    out = sg.sgmres_chebyshev_cycle(sg.DeviceCSR.from_host(A), _t(f), d, p["s"], 4.0, 4.0, 0.0, 8, 0, 0)
    ref = orc.chebyshev_cycle(A, f, d, p["s"], 8, 0, 0, 4.0, 4.0, 0.0)
    _compare_cycle(out, ref, d, 4.0, 0.0)


def test_chebyshev_full_size_converges(sg, orc):
    """n = 1,048,576, d = 200, s = 400, box [0, 8] (the spectrum of the scaled
    five-point operator): the solve reaches relative residual 1e-10."""
    A, f, p = synth.workload("cd1024")
    dA = sg.DeviceCSR.from_host(A)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    rc, info = sg.sgmres_solve(dA, _t(f), x, p["d"], 1, p["s"], p["seed"], p["tol"], p["restarts"],
                               cheb_box=(4.0, 4.0, 0.0))
    print("chebyshev full-size solve:", info, flush=True)
    assert rc == sg.OK
    _, nrm = orc.residual(A, f, _np(x))
    assert nrm / np.linalg.norm(f) <= 1e-10
