"""GPU: the differentiable solve (adjoint through the transposed sGMRES solve).

Checked against the dense FP64 adjoint gradient of the oracle and against
central finite differences of the GPU forward solve itself, on the
convection-diffusion operator at N = 32 (n = 1024).
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


def _setup(N=32):
    A = synth.convection_diffusion(N, (50.0, 20.0))
    b = synth.rhs(A.n, 0)
    xt = synth.rhs(A.n, 1)
    return A, b, xt


def test_outer_grad_kernel(sg):
    A = synth.random_dominant(5003, 6, seed=2)
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal(A.n), rng.standard_normal(A.n)
    dA = sg.DeviceCSR.from_host(A)
    out = sg.sgmres_csr_outer_grad(dA, torch.as_tensor(u, device=DEV), torch.as_tensor(v, device=DEV), -0.5)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert np.array_equal(out.cpu().numpy(), -0.5 * u[rows] * v[A.col_idx])


def test_autograd_matches_dense_gradient(sg, orc):
    A, b, xt = _setup()
    x_ref, L_ref, gb_ref, gval_ref = orc.dense_solve_gradient(A, b, xt)
    val = torch.as_tensor(A.val, device=DEV).requires_grad_(True)
    bt = torch.as_tensor(b, device=DEV).requires_grad_(True)
    rp = torch.as_tensor(A.row_ptr, device=DEV)
    ci = torch.as_tensor(A.col_idx, device=DEV)
    x = sg.sgmres_solve_diff(rp, ci, val, bt, d=200, k=4, s=400, tol=1e-13)
    L = ((x - torch.as_tensor(xt, device=DEV)) ** 2).sum()
    L.backward()
    assert np.linalg.norm(x.detach().cpu().numpy() - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    assert abs(float(L.detach()) - L_ref) <= 1e-8 * L_ref
    gb = bt.grad.cpu().numpy()
    gv = val.grad.cpu().numpy()
    assert np.linalg.norm(gb - gb_ref) <= 1e-8 * np.linalg.norm(gb_ref)
    assert np.linalg.norm(gv - gval_ref) <= 1e-8 * np.linalg.norm(gval_ref)


def test_autograd_finite_differences(sg):
    A, b, xt = _setup()
    rp = torch.as_tensor(A.row_ptr, device=DEV)
    ci = torch.as_tensor(A.col_idx, device=DEV)
    xtt = torch.as_tensor(xt, device=DEV)

    def loss(valnp, bnp, grad=False):
        val = torch.as_tensor(valnp, device=DEV).requires_grad_(grad)
        bt = torch.as_tensor(bnp, device=DEV).requires_grad_(grad)
        x = sg.sgmres_solve_diff(rp, ci, val, bt, d=200, k=4, s=400, tol=1e-14)
        L = ((x - xtt) ** 2).sum()
        if grad:
            L.backward()
            return float(L.detach()), val.grad.cpu().numpy(), bt.grad.cpu().numpy()
        return float(L)

    L0, gv, gb = loss(A.val, b, grad=True)
    rng = np.random.default_rng(3)
    for q in rng.choice(A.nnz, 6, replace=False):
        h = 1e-6 * abs(A.val[q])
        vp, vm = A.val.copy(), A.val.copy()
        vp[q] += h
        vm[q] -= h
        fd = (loss(vp, b) - loss(vm, b)) / (2 * h)
        assert abs(fd - gv[q]) <= 1e-4 * np.abs(gv).max()
    for i in rng.choice(A.n, 4, replace=False):
        h = 1e-6
        bp, bm = b.copy(), b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss(A.val, bp) - loss(A.val, bm)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-4 * np.abs(gb).max()
