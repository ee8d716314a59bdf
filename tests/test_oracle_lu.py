"""Pins of the oracle's LU factorization with partial pivoting (the paper's
LU function block, section 5.1(b)) against what the mathematics and an
independent library fix: exact rational elimination on small integer
matrices, LAPACK's getrf (scipy), the reconstruction P A = L U, the
partial-pivoting bound |L| <= 1, singular and special matrices."""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def unpack(lu, ipiv):
    n = lu.shape[0]
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    perm = np.arange(n)
    for j, p in enumerate(ipiv):
        perm[[j, p]] = perm[[p, j]]
    return L, U, perm


def exact_lu(a):
    """Gaussian elimination with partial pivoting in exact rationals; the
    pivot is the first row of largest magnitude."""
    n = len(a)
    m = [[Fraction(v) for v in row] for row in a]
    piv = []
    for j in range(n):
        p = max(range(j, n), key=lambda i: (abs(m[i][j]), -i))
        piv.append(p)
        m[j], m[p] = m[p], m[j]
        if m[j][j] == 0:
            continue
        for i in range(j + 1, n):
            m[i][j] /= m[j][j]
            for c in range(j + 1, n):
                m[i][c] -= m[i][j] * m[j][c]
    return m, piv


def test_two_by_two_by_hand():
    lu, ipiv, info = oracle.lu([[1.0, 2.0], [3.0, 4.0]])
    assert list(ipiv) == [1, 1] and info == 0
    assert lu[0].tolist() == [3.0, 4.0]
    # binary64 without contraction: l = RN(1/3), u = RN(2 - RN(l * 4))
    assert lu[1, 0] == 1.0 / 3.0 and lu[1, 1] == 2.0 - (1.0 / 3.0) * 4.0


@pytest.mark.parametrize("seed", range(12))
def test_small_integer_matrices_match_exact_elimination(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    a = rng.integers(-9, 10, size=(n, n)).astype(float)
    lu, ipiv, info = oracle.lu(a)
    m, piv = exact_lu(a.tolist())
    assert list(ipiv) == piv
    ref = np.array([[float(v) for v in row] for row in m])
    assert np.allclose(lu, ref, rtol=1e-13, atol=1e-13)
    assert info == next((j + 1 for j in range(n) if m[j][j] == 0), 0)


@pytest.mark.parametrize("n", [1, 5, 64, 200])
def test_matches_lapack_getrf(n):
    scipy_linalg = pytest.importorskip("scipy.linalg")
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n))
    lu, ipiv, info = oracle.lu(a)
    lu_ref, piv_ref = scipy_linalg.lu_factor(a)
    assert info == 0
    assert np.array_equal(ipiv, piv_ref)
    assert np.max(np.abs(lu - lu_ref)) < 1e-12 * max(1.0, np.max(np.abs(lu_ref)))


@pytest.mark.parametrize("n", [3, 33, 128, 300])
def test_reconstruction_and_pivoting_bound(n):
    rng = np.random.default_rng(100 + n)
    a = rng.uniform(-1, 1, (n, n))
    lu, ipiv, info = oracle.lu(a)
    L, U, perm = unpack(lu, ipiv)
    assert info == 0
    assert np.max(np.abs(L)) <= 1.0
    assert all(ipiv[j] >= j for j in range(n))
    r = np.linalg.norm(a[perm] - L @ U) / np.linalg.norm(a)
    assert r < 1e-15 * n


def test_identity_and_permutation():
    lu, ipiv, info = oracle.lu(np.eye(7))
    assert np.array_equal(lu, np.eye(7)) and list(ipiv) == list(range(7)) and info == 0
    p = np.eye(5)[[3, 0, 4, 1, 2]]
    lu, ipiv, info = oracle.lu(p)
    assert np.array_equal(lu, np.eye(5)) and info == 0
    L, U, perm = unpack(lu, ipiv)
    assert np.array_equal(p[perm], np.eye(5))


def test_singular_reports_first_zero_pivot():
    a = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 0.0, 1.0]])   # rank 2
    m, piv = exact_lu(a.tolist())
    want = next((j + 1 for j in range(3) if m[j][j] == 0), 0)
    lu, ipiv, info = oracle.lu(a)
    assert info == want
    z = np.zeros((4, 4))
    assert oracle.lu(z)[2] == 1
    a = np.arange(16.0).reshape(4, 4)
    a[:, 1] = 0.0
    assert oracle.lu(a)[2] == 2


def test_solves_linear_systems():
    rng = np.random.default_rng(7)
    n = 50
    a = rng.standard_normal((n, n)) + n * np.eye(n)
    x = rng.standard_normal(n)
    b = a @ x
    lu, ipiv, info = oracle.lu(a)
    L, U, perm = unpack(lu, ipiv)
    y = np.linalg.solve(L, b[perm])
    got = np.linalg.solve(U, y)
    assert np.max(np.abs(got - x)) < 1e-12
