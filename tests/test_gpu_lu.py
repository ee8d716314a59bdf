"""GPU parity of the LU function block (fb_lu_factor) against the oracle's
Gaussian elimination with partial pivoting: the same pivots, factors within
rounding, the residual P A - L U at the level of binary64 rounding, singular
matrices reported by info; sizes with ragged panels and tiles up to the
paper's 2048 x 2048."""
import numpy as np
import pytest

import oracle
from paper_2004_09883_amd import fb

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def gpu_lu(a, lda=None):
    n = a.shape[0]
    lda = lda or n
    buf = torch.zeros((n, lda), dtype=torch.float64, device="cuda")
    buf[:, :n] = torch.from_numpy(a)
    view = buf[:, :n]
    ipiv = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    fb.fb_lu_factor(view, ipiv, info)
    torch.cuda.synchronize()
    return view.cpu().numpy(), ipiv.cpu().numpy(), int(info.cpu()[0]), buf.cpu().numpy()


def residual(a, lu, ipiv):
    n = a.shape[0]
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    perm = np.arange(n)
    for j, p in enumerate(ipiv):
        perm[[j, p]] = perm[[p, j]]
    return np.linalg.norm(a[perm] - L @ U) / np.linalg.norm(a)


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 33, 100, 257, 1000, 2048])
def test_lu_matches_oracle(n):
    print(f"lu n={n}", flush=True)
    a = np.random.default_rng(n).uniform(-1, 1, (n, n))
    lu, ipiv, info, _ = gpu_lu(a)
    lu_ref, ipiv_ref, info_ref = oracle.lu(a)
    assert info == info_ref == 0
    assert np.array_equal(ipiv, ipiv_ref)
    assert np.max(np.abs(lu - lu_ref)) <= 1e-11 * np.max(np.abs(lu_ref))
    assert residual(a, lu, ipiv) < 1e-15 * n + 1e-16
    assert np.max(np.abs(np.tril(lu, -1))) <= 1.0


def test_lu_with_row_stride_keeps_padding():
    n, lda = 300, 333
    a = np.random.default_rng(5).standard_normal((n, n))
    lu, ipiv, info, buf = gpu_lu(a, lda)
    lu_ref, ipiv_ref, _ = oracle.lu(a)
    assert np.array_equal(ipiv, ipiv_ref)
    assert np.max(np.abs(lu - lu_ref)) <= 1e-11 * np.max(np.abs(lu_ref))
    assert np.all(buf[:, n:] == 0.0)   # the padding columns are not touched


@pytest.mark.parametrize("n,lda", [(1537, 1601), (2047, 2051)])
def test_lu_large_with_row_stride(n, lda):
    """Odd row strides at sizes where the rows need 3 and 4 register slots,
    the trailing strips are ragged and the last panel is short: the rows
    past the end and the padding columns are read but never written."""
    print(f"lu n={n} lda={lda}", flush=True)
    a = np.random.default_rng(n + lda).uniform(-1, 1, (n, n))
    lu, ipiv, info, buf = gpu_lu(a, lda)
    lu_ref, ipiv_ref, info_ref = oracle.lu(a)
    assert info == info_ref == 0
    assert np.array_equal(ipiv, ipiv_ref)
    assert np.max(np.abs(lu - lu_ref)) <= 1e-11 * np.max(np.abs(lu_ref))
    assert np.all(buf[:, n:] == 0.0)


def test_lu_singular_and_special_matrices():
    a = np.arange(64.0 * 64).reshape(64, 64) % 7 - 3.0
    a[:, 20] = 0.0
    lu, ipiv, info, _ = gpu_lu(a)
    _, ipiv_ref, info_ref = oracle.lu(a)
    assert info == info_ref and info > 0
    eye = np.eye(50)
    lu, ipiv, info, _ = gpu_lu(eye)
    assert np.array_equal(lu, eye) and list(ipiv) == list(range(50)) and info == 0
    perm = np.eye(40)[np.random.default_rng(1).permutation(40)]
    lu, ipiv, info, _ = gpu_lu(perm)
    assert np.array_equal(lu, np.eye(40)) and info == 0


def test_lu_rejects_bad_arguments():
    ipiv = torch.zeros(8, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    big = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda")
    with pytest.raises(fb.FbError) as e:
        fb.fb_lu_factor(big, torch.zeros(4096, dtype=torch.int32, device="cuda"), info)
    assert e.value.code == fb.FB_ERR_UNSUPPORTED_SIZE
    with pytest.raises(fb.FbError):
        fb.fb_lu_factor(torch.zeros((8, 8), dtype=torch.float64, device="cuda"), ipiv[:4], info)
