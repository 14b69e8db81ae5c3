"""The allocation-free sketch entry point (sgmres_sketch_apply_noalloc)
against sgmres_sketch_apply, through the C ABI: two calls in a row, the second
on a smaller input, each bit-identical to the allocating entry point's result
(both run the same fixed-order kernels) and close to the oracle's."""

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


def _case(sg, orc, n, s, zeta, seed, cycle):
    v = torch.as_tensor(synth.rhs(n, 21 + n % 7), device=DEV)
    g = torch.full((s,), float("nan"), dtype=torch.float64, device=DEV)
    sg.sgmres_sketch_apply_noalloc(v, g, seed, cycle, s, zeta)
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    ref_gpu = sg.sgmres_sketch_apply(v, seed, cycle, s, zeta).cpu().numpy()
    assert np.array_equal(got, ref_gpu)
    ref = orc.sketch_apply(v.cpu().numpy(), seed, cycle, s, zeta)
    mass = np.abs(v.cpu().numpy()).sum() * np.sqrt(zeta) / s
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * mass)


def test_noalloc_matches_allocating_entry_two_calls(sg, orc):
    # largest scratch use first (s = 4096 over the full 512-workgroup grid),
    # then a smaller input that leaves the first call's partials behind
    _case(sg, orc, 300001, 4096, 32, 9, 4)
    _case(sg, orc, 70001, 400, 8, 3, 0)


def test_noalloc_rejects_bad_sizes(sg):
    v = torch.ones(10, dtype=torch.float64, device=DEV)
    g = torch.zeros(4097, dtype=torch.float64, device=DEV)
    with pytest.raises(sg.SGMRESError):
        sg.sgmres_sketch_apply_noalloc(v, g, 0, 0, 4097, 8)
    with pytest.raises(sg.SGMRESError):
        sg.sgmres_sketch_apply_noalloc(v, g[:8], 0, 0, 8, 9)
