"""GPU parity of the streaming truncated-Arnoldi path (systems beyond the
resident kernels' capacity) against the CPU FP64 oracle, through the C ABI.

The streaming kernel reads the window back from the basis and forms no sketch
itself; S B is formed from the finished basis and S A B from it through the
Arnoldi relation A b_j = sum_a H[a, j] b_{j-a} + nu_j b_{j+1}, which holds to
rounding.  The oracle sketches A b_j directly, so S A B agrees to rounding, and
the solution to the method's tolerances: x to 1e-8 relative, true relative
residuals within 1e-10, the residual estimate to 1e-8 relative.  Small cases
force the path (path=PATH_STREAM) at every launch shape: m and w in registers
with 4, 8 or 16 rows per thread, or parked in HBM between phases.
"""

import os

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _host_threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 1


@pytest.fixture(scope="module")
def sg():
    import paper_2111_00113_amd as sg

    sg.lib()
    return sg


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _gpu(sg, A, f, d, k, s, seed, tol, restarts, **kw):
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    rc, info = sg.sgmres_solve(sg.DeviceCSR.from_host(A), _t(f), x, d, k, s, seed, tol, restarts, **kw)
    return rc, _np(x), info


CASES = [
    # (label, operator, d, k, s)
    ("cd64_k2", lambda: synth.convection_diffusion(64, (10.0, 10.0)), 40, 2, 80),
    ("cd37_k4_ragged", lambda: synth.convection_diffusion(37, (50.0, 20.0)), 30, 4, 60),
    ("rand_k3", lambda: synth.random_dominant(5000, 6, seed=7), 25, 3, 50),
    ("cd20_k1", lambda: synth.convection_diffusion(20, (5.0, 0.0)), 12, 1, 24),
    ("cd30_d1", lambda: synth.convection_diffusion(30, (5.0, 5.0)), 1, 4, 8),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("state", [1, 2])
def test_stream_one_cycle_matches_oracle(sg, orc, case, state):
    _, make, d, k, s = case
    A = make()
    f = synth.rhs(A.n, 2)
    rc, x, info = _gpu(sg, A, f, d, k, s, 4, 0.0, 0, path=sg.PATH_STREAM, stream_state=state)
    rc_o, x_o, info_o = orc.sgmres_solve(A, f, d=d, k=k, s=s, zeta=8, seed=4, tol=0.0, restarts=0)
    assert info["path"] == sg.PATH_STREAM and (info["launch_rows"] < 0) == (state == 2)
    assert rc == rc_o == sg.NOT_CONVERGED and info["cycles"] == 1
    assert info["d_eff_last"] == info_o["d_eff_last"]
    assert np.linalg.norm(x - x_o) / np.linalg.norm(x_o) < 1e-8
    assert abs(info["relres"] - info_o["relres"]) < 1e-10
    assert np.isclose(info["rest_est"], info_o["rest_est"], rtol=1e-8)


@pytest.fixture(scope="module")
def cd256(orc):
    A = synth.convection_diffusion(256, (50.0, 20.0))
    f = synth.rhs(A.n, 0)
    orc.set_threads(_host_threads())
    try:
        out = orc.sgmres_solve(A, f, d=60, k=4, s=120, zeta=8, seed=3, tol=0.0, restarts=0)
    finally:
        orc.set_threads(1)
    return A, f, out


@pytest.mark.parametrize("state", [1, 2])
def test_stream_launch_shapes(sg, orc, cd256, state):
    """n = 65,536: 16 tiles of 4 rows per thread in registers, or the HBM state
    over the whole chip; both against the oracle, and bitwise against each other
    (the sums have the same order in both)."""
    A, f, (rc_o, x_o, info_o) = cd256
    rc, x, info = _gpu(sg, A, f, 60, 4, 120, 3, 0.0, 0, path=sg.PATH_STREAM, stream_state=state)
    assert rc == sg.NOT_CONVERGED and info["cycles"] == 1 and info["steps"] == 60
    assert np.linalg.norm(x - x_o) / np.linalg.norm(x_o) < 1e-8
    assert abs(info["relres"] - info_o["relres"]) < 1e-10
    assert np.isclose(info["rest_est"], info_o["rest_est"], rtol=1e-8)


def test_stream_register_and_hbm_state_same_bits(sg, cd256):
    A, f, _ = cd256
    outs = [_gpu(sg, A, f, 60, 4, 120, 3, 0.0, 0, path=sg.PATH_STREAM, stream_state=st) for st in (1, 2)]
    assert np.array_equal(outs[0][1], outs[1][1])


def test_stream_repeatable_bits(sg, cd256):
    A, f, _ = cd256
    a = _gpu(sg, A, f, 60, 4, 120, 3, 0.0, 0, path=sg.PATH_STREAM)
    b = _gpu(sg, A, f, 60, 4, 120, 3, 0.0, 0, path=sg.PATH_STREAM)
    assert np.array_equal(a[1], b[1]) and a[2]["relres"] == b[2]["relres"]


@pytest.mark.parametrize("N,beta,d,k", [(64, (10.0, 10.0), 40, 2), (50, (50.0, 20.0), 60, 4)])
def test_stream_restarted_to_tolerance(sg, orc, N, beta, d, k):
    A = synth.convection_diffusion(N, beta)
    f = synth.rhs(A.n, 0)
    rc, x, info = _gpu(sg, A, f, d, k, 2 * d, 0, 1e-10, 200, path=sg.PATH_STREAM)
    rc_o, x_o, info_o = orc.sgmres_solve(A, f, d=d, k=k, s=2 * d, zeta=8, seed=0, tol=1e-10, restarts=200)
    assert rc == rc_o == sg.OK
    assert abs(info["cycles"] - info_o["cycles"]) <= 1
    _, nrm = orc.residual(A, f, x)
    assert nrm / np.linalg.norm(f) <= 1e-10


def test_stream_lucky_breakdown(sg, orc):
    # A = diag(1..n), b = e_1 + e_2: the Krylov space is invariant after two
    # columns; the basis stops there and the solution is exact
    n = 300
    A = synth.diagonal(np.arange(1.0, n + 1.0))
    f = np.zeros(n)
    f[0] = f[1] = 1.0
    rc, x, info = _gpu(sg, A, f, 10, 3, 20, 0, 1e-12, 0, path=sg.PATH_STREAM)
    rc_o, x_o, info_o = orc.sgmres_solve(A, f, d=10, k=3, s=20, zeta=8, seed=0, tol=1e-12, restarts=0)
    assert info["flags"] & sg.FLAG_BREAKDOWN and info_o["flags"] & sg.FLAG_BREAKDOWN
    assert info["steps"] == 2
    assert np.allclose(x, x_o, rtol=1e-14, atol=1e-15)


def test_stream_precisions_one_cycle(sg, orc):
    A = synth.convection_diffusion(80, (10.0, 10.0))
    f = synth.rhs(A.n, 0)
    _, x_o, info_o = orc.sgmres_solve(A, f, d=40, k=2, s=80, zeta=8, seed=0, tol=0.0, restarts=0)
    _, x32, i32 = _gpu(sg, A, f, 40, 2, 80, 0, 0.0, 0, path=sg.PATH_STREAM, precision="fp32")
    err = np.linalg.norm(x32 - x_o) / np.linalg.norm(x_o)
    print(f"stream fp32 one cycle: x error {err:.2e}, residual ratio {i32['relres'] / info_o['relres']:.7f}")
    assert err < 1e-4 and abs(i32["relres"] / info_o["relres"] - 1.0) < 1e-4
    _, xb, ib = _gpu(sg, A, f, 40, 2, 80, 0, 0.0, 0, path=sg.PATH_STREAM, precision="bf16")
    print(f"stream bf16 basis one cycle: residual ratio {ib['relres'] / info_o['relres']:.4f}")
    assert ib["relres"] < 1.1 * info_o["relres"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_stream_refinement_reaches_fp64_tolerance(sg, orc, prec):
    A = synth.convection_diffusion(96, (10.0, 10.0))
    f = synth.rhs(A.n, 0)
    rc, x, info = _gpu(sg, A, f, 40, 2, 80, 0, 1e-10, 300, path=sg.PATH_STREAM, precision=prec)
    _, nrm = orc.residual(A, f, x)
    print(f"stream {prec}: cycles {info['cycles']}, relres {nrm / np.linalg.norm(f):.3e}")
    assert rc == sg.OK and nrm / np.linalg.norm(f) <= 1e-10


def test_stream_rejects_what_it_cannot_run(sg):
    A = synth.convection_diffusion(20)
    f = synth.rhs(A.n, 0)
    with pytest.raises(sg.SGMRESError):  # window beyond four columns
        _gpu(sg, A, f, 20, 6, 40, 0, 0.0, 0, path=sg.PATH_STREAM)
    with pytest.raises(sg.SGMRESError):  # more sketch rows than the lane groups hold
        _gpu(sg, A, f, 20, 2, 1100, 0, 0.0, 0, path=sg.PATH_STREAM)
    with pytest.raises(sg.SGMRESError):  # Chebyshev basis
        _gpu(sg, A, f, 20, 2, 40, 0, 0.0, 0, path=sg.PATH_STREAM, cheb_box=(4.0, 4.0, 0.0))


# ---------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def cd2048():
    A = synth.convection_diffusion(2048, (50.0, 20.0))
    return A, synth.rhs(A.n, 0)


@pytest.fixture(scope="module")
def cd2048_oracle_cycle(orc, cd2048):
    """The oracle's first cycle at full size (about 20 s on 16 host threads)."""
    A, f = cd2048
    orc.set_threads(_host_threads())
    try:
        _, x_o, info_o = orc.sgmres_solve(A, f, d=200, k=4, s=400, zeta=8, seed=0, tol=0.0, restarts=0)
    finally:
        orc.set_threads(1)
    print("oracle one cycle:", info_o, flush=True)
    return x_o, info_o


def test_stream_full_size_one_cycle_parity(sg, cd2048, cd2048_oracle_cycle):
    """n = 4,194,304 (2048 x 2048 grid, beta = (50, 20), d = 200, k = 4,
    s = 400): the automatic path for a system beyond the resident capacity, in
    the launch shape the solve picks (16 rows per thread in registers), one
    cycle against the oracle's."""
    A, f = cd2048
    rc, x, info = _gpu(sg, A, f, 200, 4, 400, 0, 0.0, 0)
    print("gpu one cycle:", {k: info[k] for k in ("path", "launch_rows", "launch_grid", "relres", "rest_est")},
          flush=True)
    assert info["path"] == sg.PATH_STREAM and info["cycles"] == 1
    x_o, info_o = cd2048_oracle_cycle
    assert np.linalg.norm(x - x_o) / np.linalg.norm(x_o) < 1e-8
    assert abs(info["relres"] - info_o["relres"]) < 1e-10
    assert np.isclose(info["rest_est"], info_o["rest_est"], rtol=1e-8)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_stream_full_size_one_cycle_reduced_precision(sg, cd2048, cd2048_oracle_cycle, prec):
    """The FP32-arithmetic instance at full size (16 rows per thread, window
    columns 0-1 in the LDS ring and 2-3 in registers; FP32 or bfloat16 basis),
    one cycle against the oracle's FP64 cycle: the solution and the true
    residual agree to what the basis precision allows."""
    A, f = cd2048
    rc, x, info = _gpu(sg, A, f, 200, 4, 400, 0, 0.0, 0, precision=prec)
    assert info["path"] == sg.PATH_STREAM and info["cycles"] == 1 and info["launch_rows"] == 16
    x_o, info_o = cd2048_oracle_cycle
    err = np.linalg.norm(x - x_o) / np.linalg.norm(x_o)
    ratio = info["relres"] / info_o["relres"]
    print(f"cd2048 {prec} one cycle: x error {err:.3e}, residual ratio {ratio:.8f}, "
          f"gpu {info['relres']:.6e} oracle {info_o['relres']:.6e}", flush=True)
    # the kernels' sums have a fixed order, so these figures are the same on
    # every run (measured: FP32 9.8e-6 and 1 + 7e-6; bfloat16 basis 3.1e-2 and
    # 6.0, its 2^-9 storage rounding of every basis entry); the bounds leave a
    # margin for a change of rounding order
    if prec == "fp32":
        assert err < 1e-4 and abs(ratio - 1.0) < 1e-4
    else:
        assert err < 0.1 and ratio < 10.0


def test_stream_full_size_lucky_breakdown(sg, orc):
    """A = diag(1..n) at n = 4,194,304 (the 16-rows-per-thread launch) and b
    with three nonzeros: the Krylov space is invariant after three columns;
    every workgroup stops at the same step and the solution is exact."""
    n = 1 << 22
    A = synth.diagonal(np.arange(1.0, n + 1.0))
    f = np.zeros(n)
    f[[0, 5000, n - 1]] = (1.0, -2.0, 3.0)
    rc, x, info = _gpu(sg, A, f, 200, 4, 400, 0, 0.0, 0)
    assert info["path"] == sg.PATH_STREAM and info["launch_rows"] == 16
    rc_o, x_o, info_o = orc.sgmres_solve(A, f, d=200, k=4, s=400, zeta=8, seed=0, tol=0.0, restarts=0)
    assert info["flags"] & sg.FLAG_BREAKDOWN and info_o["flags"] & sg.FLAG_BREAKDOWN
    assert info["steps"] == info_o["steps"] == 3
    assert np.count_nonzero(x) == 3
    # the three-column least squares has kappa ~ 4e6 (the oracle's x is off
    # the exact f / diag(A) by 8e-11 in its smallest entry)
    assert np.allclose(x, x_o, rtol=1e-8, atol=0.0)
    assert np.allclose(x[[0, 5000, n - 1]], f[[0, 5000, n - 1]] / np.array([1.0, 5001.0, float(n)]), rtol=1e-8)


@pytest.fixture(scope="module")
def cd2040_with_oracle_cycle(orc):
    A = synth.convection_diffusion(2040, (50.0, 20.0))
    f = synth.rhs(A.n, 0)
    orc.set_threads(_host_threads())
    try:
        _, x_o, info_o = orc.sgmres_solve(A, f, d=200, k=4, s=400, zeta=8, seed=0, tol=0.0, restarts=0)
    finally:
        orc.set_threads(1)
    return A, f, x_o, info_o


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stream_ragged_last_tile_one_cycle(sg, cd2040_with_oracle_cycle, prec):
    """n = 4,161,600 (2040 x 2040 grid): 16 rows per thread in registers over
    255 tiles of 16,384 rows, the last holding 64 rows, so most of its pairs
    lie past n; one cycle against the oracle's (bounds as at n = 4,194,304)."""
    A, f, x_o, info_o = cd2040_with_oracle_cycle
    rc, x, info = _gpu(sg, A, f, 200, 4, 400, 0, 0.0, 0, precision=prec)
    assert info["path"] == sg.PATH_STREAM and info["launch_rows"] == 16 and info["launch_grid"] == 255
    err = np.linalg.norm(x - x_o) / np.linalg.norm(x_o)
    print(f"cd2040 {prec} one cycle: x error {err:.3e}, relres gpu {info['relres']:.9e} "
          f"oracle {info_o['relres']:.9e}", flush=True)
    if prec == "fp64":
        assert err < 1e-8 and abs(info["relres"] - info_o["relres"]) < 1e-10
        assert np.isclose(info["rest_est"], info_o["rest_est"], rtol=1e-8)
    else:
        assert err < 1e-4 and abs(info["relres"] / info_o["relres"] - 1.0) < 1e-4


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_stream_full_size_converges(sg, orc, cd2048, prec):
    A, f = cd2048
    rc, x, info = _gpu(sg, A, f, 200, 4, 400, 0, 1e-10, 1000, precision=prec)
    _, nrm = orc.residual(A, f, x)
    print(f"cd2048 {prec}: cycles {info['cycles']}, relres {nrm / np.linalg.norm(f):.3e}", flush=True)
    assert rc == sg.OK and info["path"] == sg.PATH_STREAM
    assert nrm / np.linalg.norm(f) <= 1e-10
    assert abs(info["relres"] - nrm / np.linalg.norm(f)) <= 1e-12
