"""GPU: the allocation-free FP64 diagnostics (cloth_reduce_fp64_noalloc) against the workspace
call cloth_reduce_fp64 through the C ABI. Both run the same kernels, so the results must agree
bit for bit; two calls in a row, the second on a smaller batch, show that partials left in the
library's fixed array by one call never reach the next. A plan beyond the array's size is refused
before any launch."""
import numpy as np
import pytest

from paper_2403_12820_amd import inputs as I
from tests.gpu_util import dev_tensor, perturbed_batch

pytestmark = pytest.mark.gpu

MAT = I.Material()


def _pair(L, torch, batch, seed, with_ref=True):
    s = dev_tensor(batch.state)
    ref = dev_tensor(batch.state + I.random_array(batch.state.shape, seed=seed, scale=1e-3).astype(np.float32)) \
        if with_ref else None
    plan = L.Plan.from_batch(batch)
    out_ws = torch.full((4 * batch.n,), float("nan"), dtype=torch.float64, device="cuda")
    out_na = torch.full((4 * batch.n,), float("nan"), dtype=torch.float64, device="cuda")
    L.cloth_reduce_fp64(plan, L.ms_params(MAT), s, ref, out_ws)
    L.cloth_reduce_fp64_noalloc(plan, L.ms_params(MAT), s, ref, out_na)
    torch.cuda.synchronize()
    plan.close()
    return out_ws.cpu().numpy(), out_na.cpu().numpy()


def test_noalloc_reduce_equals_workspace_call_twice_second_smaller():
    import torch
    from paper_2403_12820_amd import _lib as L
    print("noalloc reduce: 24 cloths of 256x256 plus ragged ones, then a small batch", flush=True)
    big = perturbed_batch([(256, 256)] * 24 + [(33, 65), (17, 23), (1, 2)], seed=31)
    small = perturbed_batch([(40, 12), (9, 20), (2, 257)], seed=32)
    for batch, seed in ((big, 41), (small, 42)):
        a, b = _pair(L, torch, batch, seed)
        assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
        np.testing.assert_array_equal(a, b)
    # without a reference state (position error 0) after the larger call
    a, b = _pair(L, torch, small, 43, with_ref=False)
    np.testing.assert_array_equal(a, b)
    assert np.all(b.reshape(-1, 4)[:, 0] == 0.0)


def test_noalloc_reduce_refuses_plans_beyond_its_array():
    import torch
    from paper_2403_12820_amd import _lib as L
    print("noalloc reduce: a plan of 513 cloths of 256x256 is refused", flush=True)
    n = 513  # 513 * 256 chunks of 256 nodes, one instance more than the array holds
    H = np.full(n, 256, np.int32)
    pin = np.zeros(n * 256 * 256, np.uint8)
    plan = L.Plan(H, H.copy(), np.full(n, 1 / 31, np.float32), np.full(n, 1 / 1024, np.float32),
                  np.zeros((n, 3), np.float32), pin)
    s = torch.zeros(16, device="cuda")
    out = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(L.PecnnError, match="allocation-free"):
        L.cloth_reduce_fp64_noalloc(plan, L.ms_params(MAT), s, None, out)
    torch.cuda.synchronize()
    assert out.cpu().numpy().tolist() == [7.0] * 4
    plan.close()
