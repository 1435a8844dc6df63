"""GPU parity of the individual kernels against the oracle (through the C ABI)."""
import numpy as np
import pytest

import synth
from oracle import teter
from oracle.hamiltonian import Operator

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("K,m,n", [(1000, 70, 37), (4096, 64, 64), (77, 5, 130), (13824, 96, 96),
                                   (13824, 144, 288), (1000, 432, 144)])
def test_gram_product_matches_numpy(dev, K, m, n):
    """C = A^T B split over K chunks; m and n multiples of 144 take the
    144 x 144 tiles."""
    from paper_1506_08147_amd import gemm_batched
    rng = np.random.default_rng(K + m)
    A = rng.standard_normal((3, m, K))   # column-major K x m per problem
    B = rng.standard_normal((3, n, K))
    C = gemm_batched(1, _t(A, dev), _t(B, dev)).cpu().numpy()
    for i in range(3):
        ref = A[i] @ B[i].T               # (m x n) = A^T B
        got = C[i].T                      # stored column-major m x n
        assert np.abs(got - ref).max() <= 1e-13 * np.sqrt(K) * 10


@pytest.mark.parametrize("K,m,n", [(1000, 70, 37), (77, 5, 130), (13824, 96, 64), (1000, 70, 144),
                                   (13824, 432, 288)])
def test_update_product_matches_numpy(dev, K, m, n):
    """Y = alpha A C + beta Y; n a multiple of 144 takes the 144-wide column
    tiles."""
    from paper_1506_08147_amd import gemm_batched
    rng = np.random.default_rng(K * 3 + n)
    A = rng.standard_normal((2, m, K))
    B = rng.standard_normal((2, n, m))    # column-major m x n
    C0 = rng.standard_normal((2, n, K))
    C = gemm_batched(0, _t(A, dev), _t(B, dev), alpha=-0.7, beta=1.3, Cin=_t(C0, dev)).cpu().numpy()
    for i in range(2):
        ref = -0.7 * (A[i].T @ B[i].T) + 1.3 * C0[i].T    # K x n
        assert np.abs(C[i].T - ref).max() <= 1e-13 * np.sqrt(m) * 10


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("K,m,n", [(1000, 70, 37), (13824, 96, 96), (13824, 144, 288),
                                   (77760, 144, 144)])
def test_gram_product_fp32_kernels(dev, K, m, n):
    """The mixed form's Gram kernels: against the FP64 product of the
    operands rounded to FP32, within the worst-case bound of FP32
    summation over K terms, gamma_K sum |a||b|; their typical error is that
    of FP32 arithmetic (far above FP64 rounding, below the random-walk
    size u sqrt(K) of a sequential FP32 sum)."""
    from paper_1506_08147_amd import gemm_batched
    rng = np.random.default_rng(K + 3 * m)
    A = rng.standard_normal((2, m, K))
    B = rng.standard_normal((2, n, K))
    C = gemm_batched(1, _t(A, dev), _t(B, dev), fp32=True).cpu().numpy()
    u = 2.0 ** -24
    gam = K * u / (1 - K * u)
    rel = []
    for i in range(2):
        ref = _f32(A[i]) @ _f32(B[i]).T
        bound = gam * (np.abs(_f32(A[i])) @ np.abs(_f32(B[i])).T)
        err = np.abs(C[i].T - ref)
        assert np.all(err <= bound)
        rel.append(np.median(err / np.sqrt(np.abs(A[i]) ** 2 @ (np.abs(B[i]) ** 2).T)))
    # below u sqrt(K), the random-walk size of sequential FP32 summation
    assert 1e-12 < max(rel) < u * np.sqrt(K), rel


@pytest.mark.parametrize("K,m,n", [(1000, 70, 37), (13824, 96, 64), (13824, 432, 144),
                                   (77760, 144, 144)])
def test_update_product_fp32_kernels(dev, K, m, n):
    """The mixed form's update kernels: Y = alpha A C + beta Y with A C in
    FP32 (bound gamma_m sum |a||c| against the rounded operands) and the
    beta term in FP64."""
    from paper_1506_08147_amd import gemm_batched
    rng = np.random.default_rng(K * 5 + n)
    A = rng.standard_normal((2, m, K))
    B = rng.standard_normal((2, n, m))
    C0 = rng.standard_normal((2, n, K))
    C = gemm_batched(0, _t(A, dev), _t(B, dev), alpha=-0.7, beta=1.3, Cin=_t(C0, dev),
                     fp32=True).cpu().numpy()
    u = 2.0 ** -24
    gam = (m + 2) * u / (1 - (m + 2) * u)
    for i in range(2):
        prod = _f32(A[i]).T @ _f32(B[i]).T
        ref = -0.7 * prod + 1.3 * C0[i].T
        bound = 0.7 * gam * (np.abs(_f32(A[i])).T @ np.abs(_f32(B[i])).T) + 1e-14 * np.abs(ref)
        assert np.all(np.abs(C[i].T - ref) <= bound)
        assert np.abs(C[i].T - (-0.7 * (A[i].T @ B[i].T) + 1.3 * C0[i].T)).max() > 1e-10


@pytest.mark.parametrize("method,n,k", [(m, n, k) for m in (0, 1) for n, k in
                                         [(1, 1), (10, 10), (96, 32), (200, 64), (384, 128),
                                          (432, 144)]] +
                         [(0, 480, 160), (0, 600, 200), (0, 768, 256), (0, 801, 267),
                          (0, 816, 272), (0, 900, 300)])
def test_small_syev_matches_lapack(dev, n, k, method):
    """Method 0 takes the one-pass tridiagonalisation in one 1024-lane
    workgroup up to n = 512 (row groups x column groups), over eight
    workgroups per matrix with one launch per Householder step for
    513 <= n <= 832 (the Rayleigh-Ritz sizes of blocks of up to 277 states;
    odd and even orders), and the three-pass form above; the
    back-transformation keeps 6, 7 or 12 rows per lane, 13 above 768."""
    from paper_1506_08147_amd import small_syev
    rng = np.random.default_rng(n)
    M = rng.standard_normal((2, n, n))
    M = M + M.transpose(0, 2, 1)
    # second matrix with a degenerate cluster
    if n >= 10:
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        d = np.sort(rng.standard_normal(n))
        d[2:6] = d[2]
        M[1] = Q @ np.diag(d) @ Q.T
    w, Z = small_syev(_t(M, dev), k, method)
    w, Z = w.cpu().numpy(), Z.cpu().numpy()
    for i in range(2):
        A = M[i]
        wr = np.linalg.eigvalsh(A)
        sc = max(1.0, np.abs(wr).max())
        nw = n if method == 1 else k
        assert np.abs(w[i][:nw] - wr[:nw]).max() <= 1e-13 * sc * n
        Zi = Z[i].T                                         # n x k
        assert np.abs(A @ Zi - Zi * w[i][:k]).max() <= 1e-12 * sc * np.sqrt(n)
        assert np.abs(Zi.T @ Zi - np.eye(k)).max() <= 1e-12 * np.sqrt(n)



@pytest.mark.parametrize("J", [180, 267, 272])
def test_small_syev_structured(dev, J):
    """Method 0 on matrices whose Householder steps meet exact zeros below the
    subdiagonal (a column with nothing to reflect): the Rayleigh-Ritz matrix
    of a step whose P block is decoupled (the middle J x J block sigma I, no
    coupling), a tridiagonal and a diagonal matrix, orders 3J."""
    from paper_1506_08147_amd import small_syev
    rng = np.random.default_rng(J)
    n = 3 * J
    A = rng.standard_normal((n, n))
    A = A + A.T
    sig = 2.0 * np.abs(np.linalg.eigvalsh(A)).max()
    A[J:2 * J, :] = 0.0
    A[:, J:2 * J] = 0.0
    A[J:2 * J, J:2 * J] = sig * np.eye(J)
    T = np.diag(rng.standard_normal(n)) + np.diag(rng.standard_normal(n - 1), 1)
    T = T + np.triu(T, 1).T
    D = np.diag(rng.standard_normal(n))
    M = np.stack([A, T, D])
    w, Z = small_syev(_t(M, dev), J, 0)
    w, Z = w.cpu().numpy(), Z.cpu().numpy()
    for i in range(3):
        wr = np.linalg.eigvalsh(M[i])[:J]
        sc = max(1.0, np.abs(wr).max())
        assert np.abs(w[i][:J] - wr).max() <= 1e-13 * sc * n
        Zi = Z[i].T
        assert np.abs(M[i] @ Zi - Zi * w[i][:J]).max() <= 1e-12 * sc * np.sqrt(n)
        assert np.abs(Zi.T @ Zi - np.eye(J)).max() <= 1e-12 * np.sqrt(n)

def _handle(els):
    from paper_1506_08147_amd import ALB
    return ALB([e.grid for e in els], [e.box for e in els], [e.n_states for e in els],
               elem_lo=[e.elem_lo for e in els], elem_hi=[e.elem_hi for e in els],
               n_alb=[e.n_alb for e in els])


def _load(h, els, dev):
    import torch
    from paper_1506_08147_amd import ALB
    V = torch.cat([torch.from_numpy(e.V) for e in els]).to(dev)
    h.set_potential(V, ALB.kb_batch([e.kb for e in els], dev))


@pytest.mark.parametrize("which", ["one_element", "slab", "odd_grid", "big_plane"])
def test_apply_h_matches_oracle(dev, which):
    if which == "one_element":
        els = [synth.single_element(seed=0)]
        cols = 5
    elif which == "slab":
        els = synth.slab_batch(1, elements=[3])
        cols = 3
    elif which == "odd_grid":
        els = [synth.single_element(seed=4, grid=(20, 30, 18), n_states=6, n_atoms=4)]
        cols = 6
    else:   # xy plane above 48 x 48 points (large-tile kernels)
        els = [synth.single_element(seed=6, grid=(60, 48, 12), n_states=5, n_atoms=5)]
        cols = 5
    # put the element of interest last, behind a different one, to exercise batching
    els = [synth.single_element(seed=9, grid=(12, 12, 12), n_states=4, n_atoms=2)] + els
    h = _handle(els)
    _load(h, els, dev)
    e = els[-1]
    op = Operator(e.grid, e.box, e.V, e.kb)
    X = e.X0[:, :cols]
    HX = h.apply_h(1, _t(X.T, dev)).cpu().numpy().T
    ref = op.apply(X)
    rel = np.abs(HX - ref).max() / np.abs(ref).max()
    print(which, "rel err", rel)
    assert rel < 1e-13
    h.close()


def test_precondition_matches_oracle(dev):
    el = synth.single_element(seed=1)
    h = _handle([el])
    _load(h, [el], dev)
    rng = np.random.default_rng(5)
    X = np.linalg.qr(el.X0[:, :7])[0]
    R = rng.standard_normal((el.ng, 7))
    W = h.precondition(0, _t(R.T, dev), _t(X.T, dev)).cpu().numpy().T
    ref = teter.precondition(R, X, el.grid, el.box)
    rel = np.abs(W - ref).max() / np.abs(ref).max()
    print("precondition rel err", rel)
    assert rel < 1e-12
    h.close()


@pytest.mark.parametrize("ta,tb,dm,dn,dk", [(0, 0, 0, 0, 0), (0, 1, 0, 0, 0), (1, 0, 0, 1, 0),
                                            (1, 0, 1, 1, 0), (0, 0, 0, 1, 1), (0, 1, 0, 1, 1),
                                            (1, 1, 1, 0, 0)])
@pytest.mark.parametrize("J,kb", [(37, 3), (64, 2), (10, 1), (128, 3)])
def test_small_gemm_matches_numpy(dev, ta, tb, dm, dn, dk, J, kb):
    from paper_1506_08147_amd import small_gemm_batched
    n = kb * J
    d = lambda c: n if c == 0 else J  # noqa: E731
    M, N, K = d(dm), d(dn), d(dk)
    rng = np.random.default_rng(M * 7 + N * 3 + K + ta + 2 * tb)
    cnt = 3
    Aop = rng.standard_normal((cnt, M, K))
    Bop = rng.standard_normal((cnt, K, N))
    C0 = rng.standard_normal((cnt, M, N))
    A = np.transpose(Aop, (0, 2, 1)) if ta else Aop        # stored matrix (rows, cols)
    B = np.transpose(Bop, (0, 2, 1)) if tb else Bop
    # column-major per problem: tensor shape (cols, rows)
    At = _t(np.transpose(A, (0, 2, 1)), dev)
    Bt = _t(np.transpose(B, (0, 2, 1)), dev)
    Ct = _t(np.transpose(C0, (0, 2, 1)), dev)
    out = small_gemm_batched(ta, tb, J, kb, dm, dn, dk, At, Bt, Ct, alpha=0.5, beta=-1.25)
    got = np.transpose(out.cpu().numpy(), (0, 2, 1))
    ref = 0.5 * np.einsum("bik,bkj->bij", Aop, Bop) - 1.25 * C0
    assert np.abs(got - ref).max() <= 1e-13 * np.sqrt(K) * 10
