"""The loss-gradient entry point that allocates nothing
(bldtt_mlp_loss_grad_noalloc) against the allocating one
(bldtt_mlp_loss_grad), through the C ABI: the same kernels on the same
inputs give bit-identical gradients and losses, on two calls in a row (the
second smaller, reusing the static work memory), at the maximum size, with
missing (NaN) targets; sizes beyond the maximum are refused."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import mlp  # noqa: E402


def _lib():
    from paper_2012_06925_amd import _lib
    return _lib


def _case(n, seed):
    rng = np.random.default_rng(seed)
    model = rng.normal(0, 0.3, mlp.N_MODEL).astype(np.float32)
    model[mlp.N_PARAMS + 4:mlp.N_PARAMS + 8] = rng.uniform(0.5, 2, 4)
    feats = rng.normal(0, 1, (n, 4)).astype(np.float32)
    tgt = rng.normal(-6, 2, (n, 11)).astype(np.float32)
    tgt[rng.random((n, 11)) < 0.05] = np.nan
    dev = lambda a: torch.from_numpy(a).cuda()
    return dev(model), dev(feats), dev(tgt)


def _both(model, feats, tgt, n):
    L = _lib()
    lib = L.lib()
    P = mlp.N_PARAMS
    outs = []
    for name in ("bldtt_mlp_loss_grad", "bldtt_mlp_loss_grad_noalloc"):
        grad = torch.full((P,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        rc = getattr(lib, name)(model.data_ptr(), feats.data_ptr(), tgt.data_ptr(), n, grad.data_ptr(),
                                loss.data_ptr(), C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == L.OK, (name, L.lib().bldtt_last_error())
        torch.cuda.synchronize()
        outs.append((grad.cpu().numpy(), float(loss.cpu().numpy()[0])))
    return outs


def test_noalloc_loss_grad_equals_allocating_entry_point_twice():
    for n, seed in ((3000, 1), (700, 2)):          # the second call is smaller
        model, feats, tgt = _case(n, seed)
        (g0, l0), (g1, l1) = _both(model, feats, tgt, n)
        assert np.all(np.isfinite(g0)) and np.isfinite(l0)
        assert np.array_equal(g0, g1) and l0 == l1, (n, np.abs(g0 - g1).max(), l0, l1)
        # and both agree with the FP64 reference of the model
        ref = mlp.grad(model.cpu().numpy().astype(np.float64), feats.cpu().numpy().astype(np.float64),
                       tgt.cpu().numpy().astype(np.float64))
        assert np.linalg.norm(g1 - ref) <= 1e-4 * np.linalg.norm(ref)


def test_noalloc_loss_grad_at_maximum_size_and_refusals():
    L = _lib()
    n = 4096
    model, feats, tgt = _case(n, 3)
    (g0, l0), (g1, l1) = _both(model, feats, tgt, n)
    assert np.array_equal(g0, g1) and l0 == l1
    grad = torch.empty(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    big = _case(n + 1, 4)
    rc = L.lib().bldtt_mlp_loss_grad_noalloc(big[0].data_ptr(), big[1].data_ptr(), big[2].data_ptr(), n + 1,
                                             grad.data_ptr(), loss.data_ptr(), None)
    assert rc == L.EINVAL
    rc = L.lib().bldtt_mlp_loss_grad_noalloc(model.data_ptr(), feats.data_ptr(), tgt.data_ptr(), 0,
                                             grad.data_ptr(), loss.data_ptr(), None)
    assert rc == L.EINVAL
