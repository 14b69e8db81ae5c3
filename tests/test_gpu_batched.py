"""Batched solve (many systems per launch) against the CPU oracle.

Each system of a batch must get what the oracle's standalone restarted sGMRES
gives for it: the same sketch (keyed by seed, cycle and the row within the
system) and the same stopping rule.  FP64 bars as for the single-system path:
x to 1e-8 relative and the true relative residual to 1e-10 absolute; the
mixed-precision batch reaches 1e-10 with FP64 refinement.  Both batched
kernels are covered: several systems per resident basis launch (the default,
PATH_MULTI) and the part-split kernel (PATH_PART_SPLIT).
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


def _mixed_batch(d):
    """Uneven sizes, several workgroup chunks, ragged tails, n = d, and both
    matrix classes."""
    mats = [
        synth.random_dominant(5000, offdiag=6, seed=[4, 0]),
        synth.random_dominant(1200, offdiag=6, seed=[4, 1]),
        synth.convection_diffusion(30, (10.0, 10.0)),
        synth.random_dominant(d, offdiag=6, seed=[4, 3]),
        synth.random_dominant(9001, offdiag=6, seed=[4, 4]),
        synth.convection_diffusion(70, (50.0, 20.0)),
    ]
    return [(A, synth.rhs(A.n, [0, i])) for i, A in enumerate(mats)]


PATHS = ["multi", "part_split"]


def _path(sg, name):
    return {"multi": sg.PATH_MULTI, "part_split": sg.PATH_PART_SPLIT}[name]


def _run(sg, batch, d, k, s, tol, restarts, **kw):
    print(f"[batched] {len(batch)} systems, n = {[A.n for A, _ in batch][:8]}, d={d} k={k} s={s} tol={tol} "
          f"restarts={restarts} {kw}", flush=True)
    dev = [(sg.DeviceCSR.from_host(A), _t(b), torch.zeros(A.n, dtype=torch.float64, device=DEV)) for A, b in batch]
    rc, res = sg.sgmres_solve_batched(dev, d, k, s, 3, tol, restarts, **kw)
    return rc, res, [_np(x) for _, _, x in dev]


@pytest.mark.parametrize("path", PATHS)
def test_batched_one_cycle_parity(sg, orc, path):
    d, k, s = 40, 2, 90
    batch = _mixed_batch(d)
    rc, res, xs = _run(sg, batch, d, k, s, 0.0, 0, path=_path(sg, path))
    assert rc == sg.NOT_CONVERGED  # tol 0: every system stops after its one cycle
    for (A, b), r, x in zip(batch, res, xs):
        rc_o, x_o, info_o = orc.sgmres_solve(A, b, d=d, k=k, s=s, zeta=8, seed=3, tol=0.0, restarts=0)
        assert r["cycles"] == 1 and r["steps"] == info_o["steps"]
        assert np.linalg.norm(x - x_o) <= 1e-8 * np.linalg.norm(x_o), A.n
        assert abs(r["relres"] - info_o["relres"]) <= 1e-10


@pytest.mark.parametrize("path", PATHS)
def test_batched_restarted_parity(sg, orc, path):
    d, k, s = 40, 2, 90
    batch = _mixed_batch(d)
    rc, res, xs = _run(sg, batch, d, k, s, 1e-10, 300, path=_path(sg, path))
    assert rc == sg.OK
    for (A, b), r, x in zip(batch, res, xs):
        rc_o, x_o, info_o = orc.sgmres_solve(A, b, d=d, k=k, s=s, zeta=8, seed=3, tol=1e-10, restarts=300)
        _, nrm = orc.residual(A, b, x)
        print(f"n={A.n}: cycles {r['cycles']} (oracle {info_o['cycles']}), relres {nrm / np.linalg.norm(b):.3e}",
              flush=True)
        assert r["status"] == sg.OK
        assert nrm / np.linalg.norm(b) <= 1e-10
        assert abs(r["cycles"] - info_o["cycles"]) <= 1
        assert np.linalg.norm(x - x_o) <= 1e-8 * np.linalg.norm(x_o)


@pytest.mark.parametrize("path", PATHS)
def test_batched_multipart_parity(sg, orc, path):
    # systems above 16384 rows (part-split kernel) or 4096 rows (multi-system
    # launch) are spread over several workgroups that synchronise per step;
    # results must match the oracle as for one workgroup
    d, k, s = 40, 2, 90
    mats = [synth.random_dominant(70001, offdiag=6, seed=[6, 0]), synth.convection_diffusion(200, (50.0, 20.0)),
            synth.random_dominant(17000, offdiag=6, seed=[6, 2]), synth.random_dominant(3000, offdiag=6, seed=[6, 3])]
    batch = [(A, synth.rhs(A.n, [1, i])) for i, A in enumerate(mats)]
    for tol, restarts in ((0.0, 0), (1e-10, 200)):
        rc, res, xs = _run(sg, batch, d, k, s, tol, restarts, path=_path(sg, path))
        for (A, b), r, x in zip(batch, res, xs):
            rc_o, x_o, info_o = orc.sgmres_solve(A, b, d=d, k=k, s=s, zeta=8, seed=3, tol=tol, restarts=restarts)
            print(f"n={A.n} tol={tol}: cycles {r['cycles']} (oracle {info_o['cycles']}), relres {r['relres']:.3e} "
                  f"(oracle {info_o['relres']:.3e})", flush=True)
            assert abs(r["cycles"] - info_o["cycles"]) <= 1
            if tol == 0.0:
                assert np.linalg.norm(x - x_o) <= 1e-8 * np.linalg.norm(x_o)
                assert abs(r["relres"] - info_o["relres"]) <= 1e-10
            else:
                _, nrm = orc.residual(A, b, x)
                assert nrm / np.linalg.norm(b) <= 1e-10


def test_batched_graph_replays_match_eager(sg, orc):
    # the captured cycle graph, replayed once per cycle, against launching the
    # same kernels directly: bitwise identical after several cycles
    d, k, s = 40, 2, 90
    batch = _mixed_batch(d)
    out = []
    for eager in (False, True, False):
        rc, res, xs = _run(sg, batch, d, k, s, 1e-12, 6, eager=eager, block_size=512, rows_per_thread=4,
                           path=sg.PATH_PART_SPLIT)
        out.append((xs, [r["relres"] for r in res], [r["cycles"] for r in res]))
    for o in out[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(o[0], out[0][0]))
        assert o[1] == out[0][1] and o[2] == out[0][2]


def test_batched_shapes_agree(sg, orc):
    # every workgroup shape of the part-split kernel solves the batch (the
    # autotuner picks among them)
    d, k, s = 40, 2, 90
    batch = _mixed_batch(d)[:3]
    ref = None
    for block, R in [(256, 4), (512, 2), (512, 4), (1024, 1), (1024, 2), (1024, 4)]:
        rc, res, xs = _run(sg, batch, d, k, s, 0.0, 0, block_size=block, rows_per_thread=R, path=sg.PATH_PART_SPLIT)
        if ref is None:
            ref = xs
        for x, xr in zip(xs, ref):
            assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr), (block, R)


def test_batched_block_of_right_hand_sides(sg, orc):
    # eight systems sharing one matrix (a block of right-hand sides)
    A = synth.random_dominant(20000, offdiag=6, seed=2)
    dA = sg.DeviceCSR.from_host(A)
    bs = [synth.rhs(A.n, [2, j]) for j in range(8)]
    xs = [torch.zeros(A.n, dtype=torch.float64, device=DEV) for _ in bs]
    rc, res = sg.sgmres_solve_batched([(dA, _t(b), x) for b, x in zip(bs, xs)], 50, 2, 100, 0, 1e-10, 100)
    assert rc == sg.OK
    for b, x, r in zip(bs, xs, res):
        rc_o, x_o, info_o = orc.sgmres_solve(A, b, d=50, k=2, s=100, zeta=8, seed=0, tol=1e-10, restarts=100)
        assert np.linalg.norm(_np(x) - x_o) <= 1e-8 * np.linalg.norm(x_o)
        assert r["cycles"] == info_o["cycles"]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batched_mixed_precision_refinement(sg, orc, prec, path):
    d, k, s = 40, 2, 90
    batch = _mixed_batch(d)
    rc, res, xs = _run(sg, batch, d, k, s, 1e-10, 300, precision=prec, path=_path(sg, path))
    assert rc == sg.OK
    for (A, b), r, x in zip(batch, res, xs):
        rc_o, x_o, info_o = orc.sgmres_solve(A, b, d=d, k=k, s=s, zeta=8, seed=3, tol=1e-10, restarts=300)
        _, nrm = orc.residual(A, b, x)
        err = np.linalg.norm(x - x_o) / np.linalg.norm(x_o)
        print(f"{prec} n={A.n}: cycles {r['cycles']} (fp64 oracle {info_o['cycles']}), "
              f"relres {nrm / np.linalg.norm(b):.3e}, |x - x64|/|x| {err:.2e}", flush=True)
        assert nrm / np.linalg.norm(b) <= 1e-10
        assert err <= 1e-6


@pytest.mark.parametrize("path", PATHS)
def test_batched_edge_cases(sg, orc, path):
    d, k, s = 20, 2, 44
    A = synth.random_dominant(3000, offdiag=6, seed=1)
    dA = sg.DeviceCSR.from_host(A)
    z = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    bad = _t(synth.rhs(A.n, 1))
    bad[7] = float("nan")
    good = _t(synth.rhs(A.n, 2))
    xs = [torch.ones(A.n, dtype=torch.float64, device=DEV) for _ in range(3)]
    rc, res = sg.sgmres_solve_batched([(dA, z, xs[0]), (dA, bad, xs[1]), (dA, good, xs[2])], d, k, s, 0, 1e-10, 50,
                                      path=_path(sg, path))
    assert rc == sg.NOT_CONVERGED
    assert res[0]["status"] == sg.OK and float(xs[0].abs().max()) == 0.0  # b = 0 gives x = 0
    assert res[1]["status"] == -5  # SGMRES_ENONFINITE for that system only
    assert res[2]["status"] == sg.OK and res[2]["relres"] <= 1e-10
    # empty batch; invalid sizes are rejected before anything runs
    assert sg.sgmres_solve_batched([], d, k, s)[0] == sg.OK
    for dd, kk, ss in [(A.n + 1, 2, 2 * A.n + 4), (20, 5, 44), (20, 2, 20)]:
        with pytest.raises(sg.SGMRESError) as e:
            sg.sgmres_solve_batched([(dA, good, xs[2])], dd, kk, ss)
        assert e.value.rc == -1


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_workload_subset(sg, orc, prec, path):
    """The first 24 systems of the many-systems workload (n in [16384, 262144],
    7 nonzeros per row, d = 100, k = 2, s = 200), FP64, and FP32 cycles with
    FP64 refinement, to 1e-10; residuals confirmed by the oracle."""
    batch = synth.batch_workload(24)
    rc, res, xs = _run(sg, batch, 100, 2, 200, 1e-10, 50, precision=prec, path=_path(sg, path))
    assert rc == sg.OK
    for (A, b), r, x in zip(batch, res, xs):
        _, nrm = orc.residual(A, b, x)
        assert nrm / np.linalg.norm(b) <= 1e-10


def test_batched_routes_large_systems_to_resident_kernels(sg, orc):
    """A system of at least 2^19 rows is solved alone by the resident kernels
    (exactly what sgmres_solve gives), the others together by the part-split
    kernel; results come back in the caller's order."""
    big = synth.convection_diffusion(740, (30.0, 10.0))  # n = 547,600
    small = synth.random_dominant(20000, offdiag=6, seed=2)
    fb, fs = synth.rhs(big.n, 5), synth.rhs(small.n, 6)
    dB, dS = sg.DeviceCSR.from_host(big), sg.DeviceCSR.from_host(small)
    xs = [torch.zeros(small.n, dtype=torch.float64, device=DEV), torch.zeros(big.n, dtype=torch.float64, device=DEV)]
    print("batch: small n=20000, big n=547600", flush=True)
    rc, res = sg.sgmres_solve_batched([(dS, _t(fs), xs[0]), (dB, _t(fb), xs[1])], 60, 2, 130, 3, 1e-10, 300)
    assert rc == sg.OK
    x1 = torch.zeros(big.n, dtype=torch.float64, device=DEV)
    rc1, info1 = sg.sgmres_solve(dB, _t(fb), x1, 60, 2, 130, 3, 1e-10, 300)
    assert rc1 == sg.OK
    assert torch.equal(xs[1], x1)
    assert res[1]["cycles"] == info1["cycles"] and res[1]["relres"] == info1["relres"]
    for (A, f), x, r in zip([(small, fs), (big, fb)], xs, res):
        _, nrm = orc.residual(A, f, _np(x))
        assert nrm / np.linalg.norm(f) <= 1e-10
        assert abs(r["relres"] - nrm / np.linalg.norm(f)) <= 1e-12


def test_multi_matches_single_system_solve_bits(sg, orc):
    """A system solved in a multi-system launch runs the resident kernel's
    cycle on its own group of workgroups, then the same pipelined least
    squares, combine and residual kernels as sgmres_solve with the same
    launch shape (1024 x 4, three barriers): x agrees bit for bit, and other
    systems in the same launch do not change it."""
    d, k, s = 40, 2, 90
    batch = _mixed_batch(d)
    rc, res, xs = _run(sg, batch, d, k, s, 1e-10, 300, path=sg.PATH_MULTI)
    alone_rc, alone_res, alone_xs = _run(sg, batch[4:5], d, k, s, 1e-10, 300, path=sg.PATH_MULTI)
    assert np.array_equal(alone_xs[0], xs[4]) and alone_res[0] == res[4]
    for (A, b), r, x in zip(batch, res, xs):
        x1 = torch.zeros(A.n, dtype=torch.float64, device=DEV)
        rc1, info = sg.sgmres_solve(sg.DeviceCSR.from_host(A), _t(b), x1, d, k, s, 3, 1e-10, 300, block_size=1024,
                                    rows_per_thread=4, halo_off=True)
        err = np.linalg.norm(_np(x1) - x) / np.linalg.norm(x)
        print(f"n={A.n}: cycles {r['cycles']} / {info['cycles']}, |x_multi - x_single|/|x| = {err:.2e}", flush=True)
        assert r["cycles"] == info["cycles"] and r["steps"] == info["steps"]
        assert np.array_equal(_np(x1), x) and r["relres"] == info["relres"]


@pytest.mark.parametrize("R", [2, 4])
def test_multi_rows_per_thread(sg, orc, R):
    """Both multi-system instances (two or four rows per thread) against the
    oracle, one cycle; the two differ only in the order of partial sums."""
    d, k, s = 40, 2, 90
    batch = _mixed_batch(d)
    rc, res, xs = _run(sg, batch, d, k, s, 0.0, 0, path=sg.PATH_MULTI, rows_per_thread=R)
    for (A, b), r, x in zip(batch, res, xs):
        rc_o, x_o, info_o = orc.sgmres_solve(A, b, d=d, k=k, s=s, zeta=8, seed=3, tol=0.0, restarts=0)
        assert r["cycles"] == 1 and r["steps"] == info_o["steps"]
        assert np.linalg.norm(x - x_o) <= 1e-8 * np.linalg.norm(x_o), A.n
        assert abs(r["relres"] - info_o["relres"]) <= 1e-10


@pytest.mark.parametrize("k", [1, 3, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_window_lengths(sg, orc, k, prec):
    """The multi-system instances for other window lengths (two window columns
    in registers for k <= 2, four for k = 3, 4; FP64 with four columns and
    four rows per thread without the column look-ahead), one cycle.  Each
    system's x equals, bit for bit, that of sgmres_solve with the same launch
    shape (1024 x 4, three barriers).  Against the oracle for k = 3, 4 (FP32:
    to the basis precision); at k = 1 the basis is far from orthogonal here
    (the oracle's kappa estimate of S A B is 2.8e9 for the 900-row system),
    so only the bits against sgmres_solve are compared."""
    d, s = 40, 90
    batch = _mixed_batch(d)
    rc, res, xs = _run(sg, batch, d, k, s, 0.0, 0, path=sg.PATH_MULTI, precision=prec)
    for (A, b), r, x in zip(batch, res, xs):
        x1 = torch.zeros(A.n, dtype=torch.float64, device=DEV)
        rc1, info = sg.sgmres_solve(sg.DeviceCSR.from_host(A), _t(b), x1, d, k, s, 3, 0.0, 0, block_size=1024,
                                    rows_per_thread=4, halo_off=True, precision=prec)
        assert r["cycles"] == 1 and info["cycles"] == 1 and r["steps"] == info["steps"]
        assert np.array_equal(_np(x1), x) and r["relres"] == info["relres"], A.n
        if k == 1:
            continue
        rc_o, x_o, info_o = orc.sgmres_solve(A, b, d=d, k=k, s=s, zeta=8, seed=3, tol=0.0, restarts=0)
        err = np.linalg.norm(x - x_o) / np.linalg.norm(x_o)
        if prec == "fp64":
            assert r["steps"] == info_o["steps"]
            assert err <= 1e-8, A.n
            assert abs(r["relres"] - info_o["relres"]) <= 1e-10
        else:
            assert err <= 1e-4, (A.n, err)
            assert r["relres"] <= info_o["relres"] + 1e-4, (A.n, r["relres"], info_o["relres"])


def test_multi_tiny_systems(sg, orc):
    """Systems of 1, 2, 3 and 5 rows next to a larger one in one multi-system
    launch (d = 1; fewer than four rows: combined on their own, the rest in
    the wave's combine launch); each against the oracle and, bit for bit,
    against sgmres_solve at the same launch shape."""
    d, k, s = 1, 1, 4
    mats = [synth.random_dominant(n, offdiag=n - 1, seed=[7, n]) for n in (1, 2, 3, 5)]
    mats.append(synth.random_dominant(3000, offdiag=6, seed=[7, 0]))
    batch = [(A, synth.rhs(A.n, [5, i])) for i, A in enumerate(mats)]
    rc, res, xs = _run(sg, batch, d, k, s, 0.0, 0, path=sg.PATH_MULTI, zeta=4)
    for (A, b), r, x in zip(batch, res, xs):
        rc_o, x_o, info_o = orc.sgmres_solve(A, b, d=d, k=k, s=s, zeta=4, seed=3, tol=0.0, restarts=0)
        assert r["cycles"] == 1
        assert np.linalg.norm(x - x_o) <= 1e-12 * np.linalg.norm(x_o), A.n
        assert abs(r["relres"] - info_o["relres"]) <= 1e-12, A.n
        x1 = torch.zeros(A.n, dtype=torch.float64, device=DEV)
        rc1, info = sg.sgmres_solve(sg.DeviceCSR.from_host(A), _t(b), x1, d, k, s, 3, 0.0, 0, zeta=4,
                                    block_size=1024, rows_per_thread=4, halo_off=True)
        assert np.array_equal(_np(x1), x) and r["relres"] == info["relres"], A.n


def test_multi_waves(sg, orc):
    """More groups than fit one launch: 40 systems of 40,000-70,000 rows (10 to
    18 workgroups of 4096 rows each, about 560 in all) run in several waves;
    each against the oracle's one cycle."""
    d, k, s = 30, 2, 70
    rng = np.random.default_rng(11)
    mats = [synth.random_dominant(int(n), offdiag=6, seed=[9, i]) for i, n in enumerate(rng.integers(40000, 70001, 40))]
    batch = [(A, synth.rhs(A.n, [3, i])) for i, A in enumerate(mats)]
    rc, res, xs = _run(sg, batch, d, k, s, 0.0, 0, path=sg.PATH_MULTI)
    for (A, b), r, x in list(zip(batch, res, xs))[::7]:
        rc_o, x_o, info_o = orc.sgmres_solve(A, b, d=d, k=k, s=s, zeta=8, seed=3, tol=0.0, restarts=0)
        assert r["cycles"] == 1
        assert np.linalg.norm(x - x_o) <= 1e-8 * np.linalg.norm(x_o), A.n
        assert abs(r["relres"] - info_o["relres"]) <= 1e-10
