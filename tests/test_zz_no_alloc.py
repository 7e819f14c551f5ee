"""The allocation-free MBAR entry point against felis_mbar (same kernels, a
workspace the caller allocated): identical free energies on two calls in a
row, the second with a smaller input, and a clear rejection of an input
whose scratch exceeds the static array."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _harmonic(K, n, seed):
    rng = np.random.default_rng(seed)
    ks = np.exp(np.linspace(0.0, np.log(2.5), K))
    x2 = np.concatenate([(rng.normal(0, 1 / np.sqrt(k), (n, 3)) ** 2).sum(1) for k in ks])
    return 0.5 * ks[:, None] * x2[None, :], np.full(K, n)


def test_mbar_noalloc_matches_workspace_form():
    if not torch.cuda.is_available():
        pytest.skip('no HIP device')
    from paper_2603_22274_amd import felis
    ctx = felis.Context(0)
    try:
        for K, n, seed in ((42, 2000, 3), (7, 300, 4)):          # the second call is smaller
            u, N = _harmonic(K, n, seed)
            ud = torch.as_tensor(u).cuda().contiguous()
            f_ws, it_ws = felis.mbar(ctx, ud, N, tol=1e-12)
            f_na, it_na = felis.mbar_noalloc(ctx, ud, N, tol=1e-12)
            assert it_na == it_ws, (K, it_na, it_ws)
            assert np.array_equal(f_na, f_ws), (K, np.abs(f_na - f_ws).max())
        # 2 states x 5,000,000 samples need ~120 MB of scratch: rejected on the host
        big = torch.zeros((2, 5_000_000), dtype=torch.float64, device='cuda')
        with pytest.raises(felis.FelisError) as e:
            felis.mbar_noalloc(ctx, big, np.array([2_500_000, 2_500_000]))
        assert e.value.code == felis.E_CAPACITY and 'scratch' in str(e.value)
        torch.cuda.synchronize()
        ctx.device_check()
    finally:
        ctx.close()
