"""The allocation-free eigensolver entry point (dgdft_small_syev_noalloc,
static device workspace) against the allocating one (dgdft_small_syev) on
the same inputs, on consecutive calls whose sizes shrink (the second call
finds the first one's contents in the shared workspace), and its size
limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sym(count, n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((count, n, n))
    return M + M.transpose(0, 2, 1)


def test_noalloc_matches_allocating_entry_on_consecutive_calls():
    import torch
    from paper_1506_08147_amd import small_syev, small_syev_noalloc
    dev = torch.device("cuda:0")
    # orders 600 (512-lane kernel) then 432 and 96 (1024-lane kernel)
    for count, n, k in [(2, 600, 200), (5, 432, 144), (3, 96, 32)]:
        M = _sym(count, n, n)
        A = torch.from_numpy(M).to(dev)
        w0, Z0 = small_syev(A, k)
        w1, Z1 = small_syev_noalloc(A, k)
        torch.cuda.synchronize()
        w0, Z0, w1, Z1 = (x.cpu().numpy() for x in (w0, Z0, w1, Z1))
        sc = max(1.0, float(np.abs(w0[:, :k]).max()))
        print(f"count {count} n {n} k {k}: max |dw| {np.abs(w1[:, :k] - w0[:, :k]).max():.2e}",
              flush=True)
        assert np.abs(w1[:, :k] - w0[:, :k]).max() <= 1e-13 * sc * n
        assert np.abs(Z1 - Z0).max() <= 1e-12 * np.sqrt(n)
        for i in range(count):
            Zi = Z1[i].T
            assert np.abs(M[i] @ Zi - Zi * w1[i][:k]).max() <= 1e-12 * sc * np.sqrt(n)


def test_noalloc_rejects_a_batch_beyond_its_workspace():
    import torch
    from paper_1506_08147_amd import DGDFTError, small_syev_noalloc
    A = torch.zeros(64, 432, 432, dtype=torch.float64, device="cuda:0")
    with pytest.raises(DGDFTError) as ex:
        small_syev_noalloc(A, 144)
    assert ex.value.code == -1 and "static workspace" in str(ex.value)
