"""Pins of the FP64 reference GEMM against facts fixed by mathematics.

Each test checks the oracle against something other than itself: a library
routine on random data, exact integer arithmetic, closed forms (identity,
rank-1), and the reference-BLAS special cases of alpha and beta.  Non-square
shapes with padded leading dimensions make a transposed operand or a wrong
stride fail.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2507_15277_amd import datagen


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (7, 5, 3), (33, 17, 65), (64, 96, 128), (128, 40, 7)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-1.5, 0.5), (0.25, -2.0)])
def test_matches_numpy_float64(M, N, K, alpha, beta):
    # Library routine: numpy's FP64 matmul on the FP32 inputs widened to FP64.
    A = datagen.uniform((90, M, N, K, 0), M, K, ld=K + 3)
    B = datagen.uniform((90, M, N, K, 1), K, N, ld=N + 5)
    C0 = datagen.uniform((90, M, N, K, 2), M, N, ld=N + 1)
    Cref, S, T = oracle.ref_gemm(A, B, alpha, beta, C0)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    want_S = A64 @ B64
    want_T = np.abs(A64) @ np.abs(B64)
    want_C = alpha * want_S + beta * C0.astype(np.float64)
    scale = K * 2.0 ** -52 * want_T + 1e-300
    assert np.all(np.abs(S - want_S) <= scale)
    assert np.all(np.abs(T - want_T) <= scale)
    assert np.all(np.abs(Cref - want_C) <= abs(alpha) * scale + 4 * 2.0 ** -52 * np.abs(want_C) + 1e-300)


def test_exact_integers():
    # Integer entries in [-8, 8]: every product and partial sum is an integer
    # far below 2^53, so FP64 must reproduce exact integer arithmetic.
    M, N, K = 37, 29, 301
    A = datagen.integers((91, 0), M, K)
    B = datagen.integers((91, 1), K, N)
    Cref, S, T = oracle.ref_gemm(A, B)
    Ai, Bi = A.astype(np.int64), B.astype(np.int64)
    assert np.array_equal(S, (Ai @ Bi).astype(np.float64))
    assert np.array_equal(T, (np.abs(Ai) @ np.abs(Bi)).astype(np.float64))
    assert np.array_equal(Cref, S)


def test_identity_left_and_right():
    n, N = 48, 23
    I = np.eye(n, dtype=np.float32)
    B = datagen.uniform((92, 1), n, N)
    Cref, _, _ = oracle.ref_gemm(I, B)
    assert np.array_equal(Cref, B.astype(np.float64))
    A = datagen.uniform((92, 0), N, n)
    Cref, _, _ = oracle.ref_gemm(A, I)
    assert np.array_equal(Cref, A.astype(np.float64))


def test_rank1_closed_form():
    # A[i,k] = a_i, B[k,j] = b_j  =>  C[i,j] = K * a_i * b_j exactly.
    M, N, K = 19, 13, 250
    a = np.arange(-9, 10, dtype=np.float32)[:M]
    b = (2.0 ** np.arange(-6, 7)).astype(np.float32)[:N]
    A = np.repeat(a[:, None], K, axis=1)
    B = np.repeat(b[None, :], K, axis=0)
    Cref, S, T = oracle.ref_gemm(A, B)
    want = K * np.outer(a.astype(np.float64), b.astype(np.float64))
    assert np.array_equal(S, want)
    assert np.array_equal(T, np.abs(want))


def test_non_square_orientation():
    # C[i,j] = sum_k A[i,k] B[k,j] with A having a single 1 at (i0,k0) and B a
    # single 1 at (k0,j0): the only non-zero of C is at (i0, j0).  A transposed
    # operand or swapped strides puts it elsewhere or drops it.
    M, N, K = 5, 7, 3
    A = np.zeros((M, K), np.float32)
    B = np.zeros((K, N), np.float32)
    A[4, 2] = 3.0
    B[2, 6] = -2.0
    Cref, _, _ = oracle.ref_gemm(A, B)
    want = np.zeros((M, N))
    want[4, 6] = -6.0
    assert np.array_equal(Cref, want)


def test_alpha_zero_does_not_read_ab():
    M, N, K = 9, 11, 13
    A = np.full((M, K), np.nan, np.float32)
    B = np.full((K, N), np.nan, np.float32)
    C0 = datagen.uniform((93, 2), M, N)
    Cref, S, T = oracle.ref_gemm(A, B, 0.0, 0.5, C0)
    assert np.array_equal(Cref, 0.5 * C0.astype(np.float64))
    assert np.all(S == 0) and np.all(T == 0)


def test_beta_zero_does_not_read_c():
    M, N, K = 9, 11, 13
    A = datagen.uniform((94, 0), M, K)
    B = datagen.uniform((94, 1), K, N)
    C0 = np.full((M, N), np.nan, np.float32)
    Cref, S, _ = oracle.ref_gemm(A, B, 2.0, 0.0, C0)
    assert np.all(np.isfinite(Cref))
    assert np.array_equal(Cref, 2.0 * S)


def test_k_zero_gives_beta_c():
    M, N = 6, 4
    A = np.zeros((M, 0), np.float32)
    B = np.zeros((0, N), np.float32)
    C0 = datagen.uniform((95, 2), M, N)
    Cref, S, T = oracle.ref_gemm(A, B, 1.0, -0.5, C0)
    assert np.array_equal(Cref, -0.5 * C0.astype(np.float64))
    assert np.all(S == 0) and np.all(T == 0)


def test_alpha_minus_one_beta_one_integers():
    M, N, K = 21, 18, 40
    A = datagen.integers((96, 0), M, K)
    B = datagen.integers((96, 1), K, N)
    C0 = datagen.integers((96, 2), M, N, -100, 100)
    Cref, _, _ = oracle.ref_gemm(A, B, -1.0, 1.0, C0)
    want = -(A.astype(np.int64) @ B.astype(np.int64)) + C0.astype(np.int64)
    assert np.array_equal(Cref, want.astype(np.float64))


def test_empty_dims():
    for (M, N, K) in [(0, 5, 3), (4, 0, 3), (0, 0, 0)]:
        A = np.zeros((M, K), np.float32)
        B = np.zeros((K, N), np.float32)
        Cref, _, _ = oracle.ref_gemm(A, B)
        assert Cref.shape == (M, N)


def test_sampled_entries_match_full():
    M, N, K = 50, 70, 90
    A = datagen.uniform((97, 0), M, K, ld=K + 2)
    B = datagen.uniform((97, 1), K, N)
    C0 = datagen.uniform((97, 2), M, N)
    Cref, S, T = oracle.ref_gemm(A, B, 1.25, 0.75, C0)
    rng = np.random.default_rng(5)
    rows = rng.integers(0, M, 200)
    cols = rng.integers(0, N, 200)
    c2, s2, t2 = oracle.ref_gemm_at(A, B, rows, cols, 1.25, 0.75, C0)
    # Same per-element summation order, so the values are identical.
    assert np.array_equal(c2, Cref[rows, cols])
    assert np.array_equal(s2, S[rows, cols])
    assert np.array_equal(t2, T[rows, cols])


def test_tolerance_form():
    # alpha = 1, beta = 0: exactly 4*K*2^-24*T.
    T = np.array([[1.0, 2.0]])
    S = np.array([[0.5, -1.0]])
    tol = oracle.gemm_tolerance(100, 1.0, 0.0, S, T)
    assert np.array_equal(tol, 4 * 100 * 2.0 ** -24 * T)
    # An FP32 accumulation of uniform data sits well inside the bound.
    M, N, K = 16, 16, 512
    A = datagen.uniform((98, 0), M, K)
    B = datagen.uniform((98, 1), K, N)
    Cref, S, T = oracle.ref_gemm(A, B)
    c32 = np.zeros((M, N), np.float32)
    for k in range(K):
        c32 += np.outer(A[:, k], B[k, :]).astype(np.float32)
    err = np.abs(c32.astype(np.float64) - Cref)
    assert np.all(err <= oracle.gemm_tolerance(K, 1.0, 0.0, S, T))
    # A dropped product term violates it.
    bad = c32.astype(np.float64) - np.outer(A[:, 0], B[0, :])
    assert np.any(np.abs(bad - Cref) > oracle.gemm_tolerance(K, 1.0, 0.0, S, T))


def test_threads_reported():
    assert oracle.threads() >= 1
    assert math.isfinite(float(oracle.threads()))
