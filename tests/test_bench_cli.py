"""bench.py on the host: more than one GPU is refused with a message and a
nonzero status, before anything touches a device; the start-block layout
with guard columns and the per-workload guard defaults."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_start_block_layout_with_guards():
    """X0 of the batch: per element its n_states seeded columns, then the
    seeded guard columns, each column contiguous (host-side layout only)."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import bench
    import synth
    els = [synth.single_element(seed=s, grid=(12, 12, 12), n_states=5, n_atoms=1) for s in (0, 1)]
    X0 = bench.start_block(els, 3, torch.device("cpu")).numpy()
    off = 0
    for k, e in enumerate(els):
        blk = X0[off:off + e.ng * 8].reshape(8, e.ng).T      # column-major ng x (5 + 3)
        assert np.array_equal(blk[:, :5], e.X0)
        assert np.array_equal(blk[:, 5:], synth.guard_columns(e.ng, 3, (k, e.n_states)))
        off += e.ng * 8
    assert off == X0.size
    assert np.array_equal(bench.start_block(els, 0, torch.device("cpu")).numpy(),
                          np.concatenate([e.X0.T.ravel() for e in els]))


def test_default_guard_columns_per_workload():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.DEFAULT_GUARD == {"slab": 16, "uneven": 16, "one": 8}
    assert (128 + bench.DEFAULT_GUARD["slab"]) % 144 == 0   # the 144-wide product tiles
