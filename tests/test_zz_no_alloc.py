"""fea_mlp_grad_noalloc (the network's BCE gradient with its workspace in a
fixed device array, for callers that cannot allocate) against fea_mlp_grad
(workspace allocated per call) on the same inputs, through the C ABI: two
calls in a row, the second on fewer samples, and the size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_2605_18052_amd import fastea

pytestmark = pytest.mark.gpu

MAX_SAMPLES = 65536  # FEA_MLP_NOALLOC_MAX_SAMPLES


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(n, seed):
    import torch
    from paper_2605_18052_amd import learned
    rng = np.random.default_rng(seed)
    feat = torch.from_numpy(rng.uniform(-1, 1, size=(n, 8)).astype(np.float32)).cuda().contiguous()
    target = torch.from_numpy((rng.uniform(size=n) < 0.7).astype(np.float32)).cuda().contiguous()
    params = torch.from_numpy(learned.he_init(seed)).cuda().contiguous()
    return feat, target, params


def _noalloc(n, feat, target, params):
    import torch
    f = fastea.lib().fea_mlp_grad_noalloc  # argument types set by the binding
    grad = torch.full((params.numel(),), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = f(0, C.c_void_p(stream), C.c_void_p(feat.data_ptr()), C.c_void_p(target.data_ptr()), n,
           C.c_void_p(params.data_ptr()), C.c_void_p(grad.data_ptr()), C.c_void_p(loss.data_ptr()))
    torch.cuda.synchronize()
    return rc, grad.cpu().numpy(), float(loss.item())


def test_noalloc_matches_allocating_entry_point_twice():
    for n, seed in ((40_000, 1), (3_001, 2)):
        feat, target, params = _inputs(n, seed)
        rc, g_na, l_na = _noalloc(n, feat, target, params)
        assert rc == fastea.FEA_OK
        l_ref, g_ref = fastea.mlp_grad(feat, target, params)
        g_ref = g_ref.cpu().numpy() if hasattr(g_ref, "cpu") else np.asarray(g_ref)
        # the same kernels in the same order: identical gradient; the mean
        # loss is the same sum scaled by 1/n instead of divided by n
        np.testing.assert_array_equal(g_na, g_ref)
        assert abs(l_na - l_ref) <= 1e-12 * abs(l_ref), (l_na, l_ref)


def test_noalloc_rejects_sizes_beyond_its_workspace():
    feat, target, params = _inputs(8, 3)
    rc, _, _ = _noalloc(MAX_SAMPLES + 1, feat, target, params)
    assert rc == fastea.FEA_EINVAL
    rc, _, _ = _noalloc(0, feat, target, params)
    assert rc == fastea.FEA_EINVAL
