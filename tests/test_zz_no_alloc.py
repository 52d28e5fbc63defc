"""The allocation-free sums (mrtfd_sums_noalloc) through the C ABI: partial
sums in the library's own device scratch, result in a caller's device array,
no synchronisation.  Checked against mrtfd_sums (workspace partials, host
result) bit for bit on two calls in a row, the second on a smaller grid, so
that partials left in the shared scratch by the first call cannot leak into
the second; with and without a reference state."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_0908_3749_amd import MRT2D, _abi
    return MRT2D, _abi, torch


def _sums_both_ways(gpu, nx, ny, ref, seed):
    MRT2D, abi, torch = gpu
    ic = synth.smooth_macro(nx, ny, seed=seed, du=0.2, dr=0.1)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, synth.rates(1e-5, s5=500, s6=700),
                         {k: synth.side("periodic") for k in synth.SIDES}, ic)
    g = MRT2D.from_problem(prob, ref=ref)
    g.init_problem(prob)
    g.step(7)
    d_out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    st = abi.lib().mrtfd_sums_noalloc(g._ctx, C.c_void_p(d_out.data_ptr()))
    assert st == abi.MRTFD_OK, abi.lib().mrtfd_last_error(g._ctx)
    g.stream.synchronize()
    got = d_out.cpu().numpy()
    host = (C.c_double * 4)()
    assert abi.lib().mrtfd_sums(g._ctx, host) == abi.MRTFD_OK
    want = np.array(host[:])
    # a NULL output is refused before anything is enqueued
    assert abi.lib().mrtfd_sums_noalloc(g._ctx, None) == abi.MRTFD_ERR_ARG
    g.close()
    return got, want


@pytest.mark.parametrize("ref", [None, (1.0, 1.0)])
def test_noalloc_sums_equal_sums_two_calls(gpu, ref):
    # 1024 x 300 nodes: the largest reduction (1024 blocks, the whole scratch)
    got1, want1 = _sums_both_ways(gpu, 1024, 300, ref, seed=3)
    print("first call", got1, want1)
    assert np.array_equal(got1, want1)
    # a smaller grid next (10 blocks): stale partials beyond them are ignored
    got2, want2 = _sums_both_ways(gpu, 70, 33, ref, seed=4)
    print("second call", got2, want2)
    assert np.array_equal(got2, want2)
    assert np.all(np.isfinite(got2))
