"""Blocks of right-hand sides sharing one matrix (sgmres_solve_batched routes
systems with the same CSR arrays and n >= 65,536 to the block solve: one
streaming basis launch per cycle for up to 32 right-hand sides, each with its
own basis), against the CPU oracle's standalone solve of every right-hand side.

S A B comes from S B through the Arnoldi relation (to rounding), so the bars
are the method's tolerances: x to 1e-8 relative after one cycle, true
relative residuals within 1e-10, cycles of a restarted solve within one of the
oracle's, final residuals confirmed by the oracle's residual.
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


@pytest.fixture(scope="module")
def rd70k():
    return synth.random_dominant(70000, offdiag=6, seed=9)


def _block(sg, A, bs, d, k, s, tol, restarts, **kw):
    dA = sg.DeviceCSR.from_host(A)
    xs = [torch.zeros(A.n, dtype=torch.float64, device=DEV) for _ in bs]
    print(f"[block] {len(bs)} right-hand sides, n={A.n}, d={d} k={k} s={s} tol={tol} {kw}", flush=True)
    rc, res = sg.sgmres_solve_batched([(dA, _t(b), x) for b, x in zip(bs, xs)], d, k, s, 0, tol, restarts, **kw)
    return rc, res, [_np(x) for x in xs]


@pytest.mark.parametrize("nb", [32, 5])
def test_block_one_cycle_matches_oracle(sg, orc, rd70k, nb):
    A = rd70k
    bs = [synth.rhs(A.n, [11, j]) for j in range(nb)]
    rc, res, xs = _block(sg, A, bs, 30, 2, 60, 0.0, 0)
    assert rc == sg.NOT_CONVERGED
    orc.set_threads(_host_threads())
    try:
        for j in (0, 1, nb - 1) if nb > 3 else range(nb):
            rc_o, x_o, info_o = orc.sgmres_solve(A, bs[j], d=30, k=2, s=60, zeta=8, seed=0, tol=0.0, restarts=0)
            assert res[j]["cycles"] == 1 and res[j]["steps"] == 30
            assert np.linalg.norm(xs[j] - x_o) / np.linalg.norm(x_o) < 1e-8, j
            _, nrm = orc.residual(A, bs[j], xs[j])
            assert abs(nrm / np.linalg.norm(bs[j]) - info_o["relres"]) < 1e-10
            assert abs(res[j]["relres"] - info_o["relres"]) < 1e-10
    finally:
        orc.set_threads(1)


def test_block_matches_per_system_path(sg, rd70k):
    """The same block through the per-system kernels (path = part-split): the
    solutions agree to the method's tolerance."""
    A = rd70k
    bs = [synth.rhs(A.n, [12, j]) for j in range(6)]
    _, r1, x1 = _block(sg, A, bs, 30, 2, 60, 0.0, 0)
    _, r2, x2 = _block(sg, A, bs, 30, 2, 60, 0.0, 0, path=sg.PATH_PART_SPLIT)
    for a, b in zip(x1, x2):
        assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)


def test_block_restarted_to_tolerance(sg, orc):
    A = synth.convection_diffusion(300, (50.0, 20.0))  # n = 90,000
    bs = [synth.rhs(A.n, [13, j]) for j in range(4)]
    rc, res, xs = _block(sg, A, bs, 60, 4, 120, 1e-10, 200)
    assert rc == sg.OK
    orc.set_threads(_host_threads())
    try:
        for j in (0, 3):
            rc_o, x_o, info_o = orc.sgmres_solve(A, bs[j], d=60, k=4, s=120, zeta=8, seed=0, tol=1e-10, restarts=200)
            assert rc_o == 0 and abs(res[j]["cycles"] - info_o["cycles"]) <= 1
    finally:
        orc.set_threads(1)
    for b, x, r in zip(bs, xs, res):
        _, nrm = orc.residual(A, b, x)
        assert nrm / np.linalg.norm(b) <= 1e-10
        assert abs(r["relres"] - nrm / np.linalg.norm(b)) <= 1e-12


def test_block_edge_cases(sg, orc, rd70k):
    """b = 0 gives x = 0; a NaN in one right-hand side fails that one only;
    33 right-hand sides make a block of 32 and a block of one."""
    A = rd70k
    dA = sg.DeviceCSR.from_host(A)
    bs = [_t(synth.rhs(A.n, [14, j])) for j in range(33)]
    bs[3] = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    bs[7] = bs[7].clone()
    bs[7][5] = float("nan")
    xs = [torch.ones(A.n, dtype=torch.float64, device=DEV) for _ in bs]
    rc, res = sg.sgmres_solve_batched([(dA, b, x) for b, x in zip(bs, xs)], 30, 2, 60, 0, 1e-10, 50)
    assert rc == sg.NOT_CONVERGED
    assert res[3]["status"] == sg.OK and float(xs[3].abs().max()) == 0.0
    assert res[7]["status"] == -5
    for j in (0, 31, 32):
        assert res[j]["status"] == sg.OK
        _, nrm = orc.residual(A, _np(bs[j]), _np(xs[j]))
        assert nrm / np.linalg.norm(_np(bs[j])) <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_block_mixed_precision_refinement(sg, orc, rd70k, prec):
    A = rd70k
    bs = [synth.rhs(A.n, [15, j]) for j in range(8)]
    rc, res, xs = _block(sg, A, bs, 30, 2, 60, 1e-10, 100, precision=prec)
    assert rc == sg.OK
    for b, x, r in zip(bs, xs, res):
        _, nrm = orc.residual(A, b, x)
        assert nrm / np.linalg.norm(b) <= 1e-10
    print(f"block {prec}: cycles {[r['cycles'] for r in res]}")
