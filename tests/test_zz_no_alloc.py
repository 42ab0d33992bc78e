"""The allocation-free bias gradient (lbm_nn_bias_grad_noalloc) against
lbm_nn_bias_grad, which takes its scratch from the caller: bitwise equal
results on two calls in a row, the second with a smaller input, and the
size limit rejected with LBM_ERR_ARG."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _bias(lib, dY, scratch):
    import torch

    c, P = dY.shape
    db = torch.empty(c, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = lib.lbm_nn_bias_grad(dY.data_ptr(), c, P, db.data_ptr(), scratch.data_ptr(), st)
    assert rc == 0
    return db


def _bias_noalloc(lib, dY):
    import torch

    c, P = dY.shape
    db = torch.empty(c, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = lib.lbm_nn_bias_grad_noalloc(dY.data_ptr(), c, P, db.data_ptr(), st)
    assert rc == 0
    return db


def test_bias_grad_noalloc_matches_bias_grad_on_two_calls():
    import torch

    from paper_2506_17713_amd import nn

    lib = nn.load()
    g = torch.Generator(device="cpu").manual_seed(5)
    big = torch.randn(1000, 70001, generator=g).to("cuda")
    small = torch.randn(3, 517, generator=g).to("cuda")
    scratch = torch.empty(64 * 1000, dtype=torch.float64, device="cuda")
    for dY in (big, small):
        ref = _bias(lib, dY, scratch)
        got = _bias_noalloc(lib, dY)
        torch.cuda.synchronize()
        assert torch.equal(ref, got)
        exact = dY.double().sum(1).float()
        assert torch.allclose(got, exact, rtol=1e-6, atol=1e-6)
    # the second call was smaller: its result must not carry partials of the first
    assert np.isfinite(got.cpu().numpy()).all()


def test_bias_grad_noalloc_rejects_oversize():
    import torch

    from paper_2506_17713_amd import nn

    lib = nn.load()
    dY = torch.zeros(1025, 4, dtype=torch.float32, device="cuda")
    db = torch.empty(1025, dtype=torch.float32, device="cuda")
    rc = lib.lbm_nn_bias_grad_noalloc(dY.data_ptr(), 1025, 4, db.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)
    assert rc == -1
    rc = lib.lbm_nn_bias_grad_noalloc(None, 4, 4, db.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == -1
