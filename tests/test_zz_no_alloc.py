"""gsta_l1_loss_noalloc (the L1 loss for callers that cannot allocate)
against gsta_l1_loss through the C ABI: dL/dimage and both sums bit for bit,
on two calls in a row, the second with a smaller input."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_l1_equals_context_l1_on_two_calls():
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd import _lib
    L = _lib.load()
    ctx = G.Context(16, 1, 16, 16, 16)
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(3)
    for shape in [(2, 3, 480, 640), (1, 3, 37, 50)]:
        print(f"noalloc l1 shape {shape}", flush=True)
        img = torch.from_numpy((rng.random(shape) * 1.4 - 0.2).astype(np.float32)).cuda()
        tgt = torch.from_numpy(rng.random(shape).astype(np.float32)).cuda()
        img.view(-1)[::97] = tgt.view(-1)[::97]          # exact ties: sign(0) = 0
        n = img.numel()
        dl_ref = torch.full_like(img, float("nan"))
        dl_new = torch.full_like(img, float("nan"))
        s_ref = torch.zeros(2, dtype=torch.float64, device="cuda")
        s_new = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.l1_loss(img, tgt, dl_ref, s_ref)
        st = L.gsta_l1_loss_noalloc(img.data_ptr(), tgt.data_ptr(), n, dl_new.data_ptr(), s_new.data_ptr(),
                                    stream)
        assert st == _lib.GSTA_OK, L.gsta_last_error(None)
        torch.cuda.synchronize()
        assert torch.equal(dl_ref, dl_new)
        assert torch.equal(s_ref, s_new)
        d = (img - tgt).double()            # the loss takes the float32 difference
        assert s_new[0].item() == pytest.approx(d.abs().sum().item(), rel=1e-12)
    assert ctx.check()[0] == _lib.GSTA_OK


def test_noalloc_l1_rejects_sizes_beyond_its_maximum():
    from paper_2504_06716_amd import _lib
    L = _lib.load()
    p = ctypes.c_void_p(16)          # never dereferenced: the call is rejected first
    for count in (0, -5, _lib.L1_NOALLOC_MAX_COUNT + 1):
        assert L.gsta_l1_loss_noalloc(p, p, count, p, p, None) == _lib.GSTA_ERR_INVALID
        assert b"count" in L.gsta_last_error(None)
    assert L.gsta_l1_loss_noalloc(None, p, 100, p, p, None) == _lib.GSTA_ERR_INVALID
    assert b"NULL" in L.gsta_last_error(None)
