"""GPU parity: every compiled variant against the FP64 oracle, through the C ABI.

Bars: the elementwise bound 4*K*2^-24*|alpha|*(|A||B|) (plus the epilogue
rounding term when alpha != 1 or beta != 0, from oracle.gemm_tolerance);
bitwise equality wherever the exact result is an FP32-representable integer
reached through integer partial sums below 2^24; guard bands and padding
columns of C untouched; NaN planted where the method must not read.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2507_15277_amd import abi, datagen, space
from tests.gpu_util import GuardedC, run_gemm

pytestmark = pytest.mark.gpu

PKG = os.path.dirname(abi.LIB_PATH)
VARIANT_DIR = os.path.join(PKG, "variants")


def _manifest(prec=0):
    """(id, name) of the manifest's variants of one precision form."""
    out = []
    for line in open(os.path.join(VARIANT_DIR, "manifest.txt")):
        if not line.startswith("#"):
            f = line.split()
            if int(f[13]) == prec:
                out.append((int(f[0]), f[1]))
    return out


@pytest.fixture(scope="module")
def loaded():
    """The FP32 variants (the split-precision forms have their own tests)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = abi.variant_manifest_load(VARIANT_DIR)
    assert n == sum(len(_manifest(p)) for p in range(len(abi.FORM_NAMES)))
    return _manifest(0)


def _check(C, A, B, C0, alpha, beta, label=""):
    K = A.shape[1]
    Cref, S, T = oracle.ref_gemm(A, B, alpha, beta, C0)
    tol = oracle.gemm_tolerance(K, alpha, beta, S, T, C0)
    err = np.abs(C.astype(np.float64) - Cref)
    bad = ~(err <= tol)
    assert not bad.any(), (f"{label}: {int(bad.sum())} elements out of bound; max err/tol "
                           f"{np.max(err / np.maximum(tol, 1e-300)):.3g}")
    return float(np.max(np.where(tol > 0, err / np.maximum(tol, 1e-300), 0.0)))


def test_default_variant_first_workload(loaded):
    # 256^3, uniform [-1,1), alpha=1, beta=0, the fixed 64x64 / K-step 16 variant.
    vid = [i for i, n in loaded if n == space.DEFAULT.name][0]
    assert vid == 0
    M = N = K = 256
    A, B, _ = datagen.gemm_operands(1, M, N, K)
    C, guard = run_gemm(vid, A, B, None, 1.0, 0.0)
    assert guard
    # alpha=1, beta=0: exactly the bound 4*K*2^-24*(|A||B|)_ij.
    Cref, S, T = oracle.ref_gemm(A, B)
    assert np.all(np.abs(C - Cref) <= 4 * K * 2.0 ** -24 * T)


@pytest.mark.parametrize("shape", [(133, 97, 75), (64, 64, 16), (1, 1, 1), (257, 33, 129), (70, 6, 37)])
def test_every_variant_ragged_padded(loaded, shape):
    # Ragged sizes over several tiles, leading dimensions larger than the
    # widths (padding is NaN), alpha/beta both active.  70 x 6 x 37: N below
    # one tile and not a multiple of 4 (the load vector straddling N is the
    # tile's second), K inside one slab of most variants and not a multiple
    # of 4 (element-wise last slab).
    M, N, K = shape
    lda, ldb, ldc = K + 3, N + 5, N + 2
    A = datagen.uniform((20, M, N, K, 0), M, K)
    B = datagen.uniform((20, M, N, K, 1), K, N)
    C0 = datagen.uniform((20, M, N, K, 2), M, N)
    fails = []
    for vid, name in loaded:
        C, guard = run_gemm(vid, A, B, C0, 1.5, -0.5, lda, ldb, ldc)
        try:
            _check(C, A, B, C0, 1.5, -0.5, name)
            assert guard, f"{name}: wrote outside C"
        except AssertionError as e:
            fails.append(str(e))
    assert not fails, "\n".join(fails[:10])


def test_every_variant_vector_path(loaded):
    # Sizes and leading dimensions that are multiples of 4 with aligned bases:
    # the vector-load kernel of each variant runs.
    M, N, K = 200, 328, 136
    A, B, C0 = datagen.gemm_operands(21, M, N, K, beta=0.25)
    fails = []
    for vid, name in loaded:
        C, guard = run_gemm(vid, A, B, C0, 1.0, 0.25)
        try:
            _check(C, A, B, C0, 1.0, 0.25, name)
            assert guard, f"{name}: wrote outside C"
        except AssertionError as e:
            fails.append(str(e))
    assert not fails, "\n".join(fails[:10])


def test_every_variant_vector_path_padded(loaded):
    # The vector kernel's conditions (sizes and leading dimensions multiples
    # of 4) with NaN in the padding of every operand and K ragged against
    # every K-step: a slab unit past K that reached LDS (load-to-LDS staging
    # copies whole 16-byte units) would turn every element of C into NaN.
    M, N, K = 200, 328, 132
    lda, ldb, ldc = K + 4, N + 8, N + 4
    A = datagen.uniform((24, M, N, K, 0), M, K)
    B = datagen.uniform((24, M, N, K, 1), K, N)
    C0 = datagen.uniform((24, M, N, K, 2), M, N)
    fails = []
    for vid, name in loaded:
        C, guard = run_gemm(vid, A, B, C0, 1.5, -0.5, lda, ldb, ldc)
        try:
            _check(C, A, B, C0, 1.5, -0.5, name)
            assert guard, f"{name}: wrote outside C"
        except AssertionError as e:
            fails.append(str(e))
    assert not fails, "\n".join(fails[:10])


def _offset_matrix(a, ld):
    """(rows x ld) matrix holding `a`, NaN in the padding, starting one float
    into its buffer (4-byte but not 16-byte aligned): (tensor, address)."""
    rows, cols = a.shape
    flat = np.full(1 + rows * ld + 1, np.nan, np.float32)
    flat[1:1 + rows * ld].reshape(rows, ld)[:, :cols] = a
    t = torch.from_numpy(flat).cuda()
    return t, t.data_ptr() + 4


def test_every_variant_unaligned_rows_and_k_tail(loaded):
    # N a multiple of 4 but K not, odd leading dimensions and base addresses
    # one float past 16-byte alignment: the register-staged vector kernels
    # load whole rows in (4-byte aligned) vectors here, and the last slab,
    # which ends inside a load vector, element by element.  NaN in every
    # operand's padding and one float past its end must not reach C.
    M, N, K = 200, 328, 133
    lda, ldb, ldc = K + 2, N + 1, N + 4
    A = datagen.uniform((29, M, N, K, 0), M, K)
    B = datagen.uniform((29, M, N, K, 1), K, N)
    C0 = datagen.uniform((29, M, N, K, 2), M, N)
    tA, pA = _offset_matrix(A, lda)
    tB, pB = _offset_matrix(B, ldb)
    fails = []
    for vid, name in loaded:
        gc = GuardedC(C0, M, N, ldc)
        abi.sgemm_variant(vid, M, N, K, 1.5, pA, lda, pB, ldb, -0.5, gc.ptr, ldc)
        torch.cuda.synchronize()
        C, flat = gc.result()
        try:
            _check(C, A, B, C0, 1.5, -0.5, name)
            assert gc.untouched_outside(flat), f"{name}: wrote outside C"
        except AssertionError as e:
            fails.append(str(e))
    assert not fails, "\n".join(fails[:10])


def test_every_variant_interior_tiles(loaded):
    # 520 x 520 x 256 with padded leading dimensions (multiples of 4, NaN in
    # the padding): two whole 256-row tile rows and columns, every K-step
    # dividing K, so even the 256-wide tiles get interior work-groups that run
    # the unmasked loop, beside the edge tiles of the last 8 rows and columns.
    M, N, K = 520, 520, 256
    lda, ldb, ldc = K + 4, N + 8, N + 4
    A = datagen.uniform((25, M, N, K, 0), M, K)
    B = datagen.uniform((25, M, N, K, 1), K, N)
    C0 = datagen.uniform((25, M, N, K, 2), M, N)
    fails = []
    for vid, name in loaded:
        C, guard = run_gemm(vid, A, B, C0, 1.0, 0.5, lda, ldb, ldc)
        try:
            _check(C, A, B, C0, 1.0, 0.5, name)
            assert guard, f"{name}: wrote outside C"
        except AssertionError as e:
            fails.append(str(e))
    assert not fails, "\n".join(fails[:10])


def test_every_variant_integers_bitwise(loaded):
    # Integer entries in [-8, 8], K = 260: partial sums stay below 2^24, so
    # every variant must reproduce the exact integer result bit for bit.
    M, N, K = 97, 140, 260
    A = datagen.integers((22, 0), M, K)
    B = datagen.integers((22, 1), K, N)
    Cref, _, _ = oracle.ref_gemm(A, B)
    fails = []
    for vid, name in loaded:
        C, guard = run_gemm(vid, A, B, None, 1.0, 0.0)
        if not (np.array_equal(C.astype(np.float64), Cref) and guard):
            fails.append(name)
    assert not fails, fails[:10]


def test_identity_and_rank1(loaded):
    n, N = 96, 80
    I = np.eye(n, dtype=np.float32)
    Bm = datagen.uniform((23, 1), n, N)
    a = np.arange(-7, 8, dtype=np.float32)[np.arange(70) % 15]
    b = (2.0 ** (np.arange(50) % 9 - 4)).astype(np.float32)
    K1 = 300
    A1 = np.repeat(a[:, None], K1, axis=1)
    B1 = np.repeat(b[None, :], K1, axis=0)
    want1 = (K1 * np.outer(a.astype(np.float64), b.astype(np.float64)))
    for vid, name in loaded[:: max(1, len(loaded) // 40)]:
        C, _ = run_gemm(vid, I, Bm, None, 1.0, 0.0)
        assert np.array_equal(C, Bm), name
        C, _ = run_gemm(vid, A1, B1, None, 1.0, 0.0)
        assert np.array_equal(C.astype(np.float64), want1), name


def test_alpha_beta_special_cases(loaded):
    vid = 0
    M, N, K = 70, 50, 40
    nanA = np.full((M, K), np.nan, np.float32)
    nanB = np.full((K, N), np.nan, np.float32)
    C0 = datagen.uniform((24, 2), M, N)
    # alpha = 0: A and B are not read; C = beta*C0 exactly for beta = 2^-1.
    C, guard = run_gemm(vid, nanA, nanB, C0, 0.0, 0.5)
    assert np.array_equal(C, C0 * np.float32(0.5)) and guard
    # alpha = 0, beta = 0: zeros, C not read.
    C, guard = run_gemm(vid, nanA, nanB, np.full((M, N), np.nan, np.float32), 0.0, 0.0)
    assert np.array_equal(C, np.zeros((M, N), np.float32)) and guard
    # beta = 0: NaN in C must not propagate.
    A = datagen.uniform((24, 0), M, K)
    B = datagen.uniform((24, 1), K, N)
    C, guard = run_gemm(vid, A, B, np.full((M, N), np.nan, np.float32), 1.0, 0.0)
    assert np.all(np.isfinite(C)) and guard
    _check(C, A, B, None, 1.0, 0.0)
    # K = 0: C = beta*C0.
    C, guard = run_gemm(vid, np.zeros((M, 0), np.float32), np.zeros((0, N), np.float32), C0, 1.0, -2.0,
                        lda=1, ldb=N)
    assert np.array_equal(C, C0 * np.float32(-2.0)) and guard
    # alpha = -1, beta = 1 on integers: exact.
    Ai = datagen.integers((24, 3), M, K)
    Bi = datagen.integers((24, 4), K, N)
    Ci = datagen.integers((24, 5), M, N, -50, 50)
    C, guard = run_gemm(vid, Ai, Bi, Ci, -1.0, 1.0)
    want = -(Ai.astype(np.int64) @ Bi.astype(np.int64)) + Ci.astype(np.int64)
    assert np.array_equal(C.astype(np.int64), want) and guard


def test_empty_problem_leaves_c_untouched(loaded):
    for (M, N, K) in [(0, 8, 8), (8, 0, 8)]:
        A = np.ones((M, K), np.float32)
        B = np.ones((K, N), np.float32)
        C, guard = run_gemm(0, A, B, None, 1.0, 0.0, lda=K, ldb=max(N, 1), ldc=max(N, 1))
        assert guard


def test_deterministic(loaded):
    M, N, K = 300, 260, 520
    A, B, _ = datagen.gemm_operands(25, M, N, K)
    for vid, name in loaded[:: max(1, len(loaded) // 25)]:
        C1, _ = run_gemm(vid, A, B, None, 1.0, 0.0)
        C2, _ = run_gemm(vid, A, B, None, 1.0, 0.0)
        assert np.array_equal(C1, C2), name


def test_screen_kernels_agree_with_oracle(loaded):
    M, N, K = 150, 130, 170
    A, B, C0 = datagen.gemm_operands(26, M, N, K, beta=0.5)
    dA = torch.from_numpy(A.copy()).cuda()
    dB = torch.from_numpy(B.copy()).cuda()
    dC0 = torch.from_numpy(C0.copy()).cuda()
    ref = torch.empty(M * N, dtype=torch.float64, device="cuda")
    tol = torch.empty(M * N, dtype=torch.float64, device="cuda")
    abi.screen_reference(M, N, K, 1.0, dA, K, dB, N, 0.5, dC0, N, ref, tol)
    Cref, S, T = oracle.ref_gemm(A, B, 1.0, 0.5, C0)
    r = ref.cpu().numpy().reshape(M, N)
    assert np.allclose(r, Cref, rtol=0, atol=1e-12)
    tl = tol.cpu().numpy().reshape(M, N)
    assert np.allclose(tl, oracle.gemm_tolerance(K, 1.0, 0.5, S, T, C0), rtol=1e-12, atol=0)
    dC = dC0.clone()
    abi.sgemm_variant(0, M, N, K, 1.0, dA, K, dB, N, 0.5, dC, N)
    nbad, ratio = abi.screen_compare(M, N, dC, N, ref, tol)
    assert nbad == 0 and ratio < 1.0
    dC[3, 4] += 1.0                        # a planted wrong element is caught
    nbad, ratio = abi.screen_compare(M, N, dC, N, ref, tol)
    assert nbad == 1 and ratio > 1.0


def _split_variants(loaded):
    out = []
    for vid, name in loaded:
        desc = abi.variant_info(vid).split()
        if int(desc[12]) > 1:
            out.append((vid, name))
    return out


def test_k_split_variants_long_k(loaded):
    # Long K over few tiles: every K-split variant splits here.  Two calls in
    # a row must both be right (each call rewrites every slice of partial
    # products it reduces) and bitwise equal (partials are summed in a fixed
    # order).
    M, N, K = 96, 80, 2000
    A, B, C0 = datagen.gemm_operands(27, M, N, K, beta=0.75)
    splits = _split_variants(loaded)
    assert splits
    fails = []
    for vid, name in splits:
        C1, g1 = run_gemm(vid, A, B, C0, 1.0, 0.75)
        C2, g2 = run_gemm(vid, A, B, C0, 1.0, 0.75)
        try:
            _check(C1, A, B, C0, 1.0, 0.75, name)
            assert g1 and g2, f"{name}: wrote outside C"
            assert np.array_equal(C1, C2), f"{name}: not deterministic"
        except AssertionError as e:
            fails.append(str(e))
    assert not fails, "\n".join(fails[:10])


def test_k_split_integers_and_nan_c(loaded):
    # Exact integers through the split path; beta = 0 with NaN C.
    M, N, K = 70, 130, 1500
    A = datagen.integers((28, 0), M, K, -4, 4)
    B = datagen.integers((28, 1), K, N, -4, 4)
    Cref, _, _ = oracle.ref_gemm(A, B)
    nanC = np.full((M, N), np.nan, np.float32)
    fails = []
    for vid, name in _split_variants(loaded):
        C, guard = run_gemm(vid, A, B, nanC, 1.0, 0.0)
        if not (np.array_equal(C.astype(np.float64), Cref) and guard):
            fails.append(name)
    assert not fails, fails[:10]
