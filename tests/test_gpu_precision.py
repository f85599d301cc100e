"""GPU parity of the split-precision forms (bf16x3, bf16x6, scaled fp16).

Each variant's result is compared with the oracle's exact value of the same
form (the 16-bit pieces formed by definition, their kept products summed in
FP64): the difference may only be FP32 accumulation of the term products,
bounded like the FP32 GEMM's.  The error against the true product is
checked against the form's truncation bound."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import precision_ref as pr
from paper_2507_15277_amd import abi, datagen, tuned
from tests.gpu_util import run_gemm

pytestmark = pytest.mark.gpu

VARIANT_DIR = tuned.VARIANT_DIR
FORMS = {1: "bf16x3", 2: "bf16x6", 3: "fp16s", 4: "fp16x3"}
SCALED = ("fp16s", "fp16x3")     # forms with the per-matrix power-of-two scale


def _split_variants():
    out = []
    for line in open(os.path.join(VARIANT_DIR, "manifest.txt")):
        if not line.startswith("#"):
            f = line.split()
            if int(f[13]) > 0:
                out.append((int(f[0]), f[1], FORMS[int(f[13])]))
    return out


@pytest.fixture(scope="module")
def split_loaded():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.variant_manifest_load(VARIANT_DIR)
    v = _split_variants()
    assert {f for _, _, f in v} == set(FORMS.values())
    return v


def _check_form(C, A, B, form, alpha=1.0, beta=0.0, C0=None, label=""):
    K = A.shape[1]
    Cs, Ts = pr.split_form_gemm(A, B, form, alpha, beta, C0)
    tol = pr.accumulation_tolerance(K, form, alpha, beta, Ts, Cs, C0)
    err = np.abs(C.astype(np.float64) - Cs)
    bad = ~(err <= tol)
    assert not bad.any(), (f"{label}: {int(bad.sum())} elements off the {form} value; max err/tol "
                           f"{np.max(err / np.maximum(tol, 1e-300)):.3g}")


@pytest.mark.parametrize("shape,lds", [((133, 97, 75), (3, 5, 2)), ((200, 328, 136), (0, 0, 0)),
                                       ((1, 1, 1), (0, 0, 0)), ((70, 300, 520), (4, 0, 4))])
def test_split_forms_match_oracle(split_loaded, shape, lds):
    M, N, K = shape
    lda, ldb, ldc = K + lds[0], N + lds[1], N + lds[2]
    A = datagen.lognormal((40, M, N, K, 0), M, K)
    B = datagen.lognormal((40, M, N, K, 1), K, N)
    C0 = datagen.uniform((40, M, N, K, 2), M, N)
    fails = []
    for vid, name, form in split_loaded:
        C, guard = run_gemm(vid, A, B, C0, 1.5, -0.5, lda, ldb, ldc)
        try:
            _check_form(C, A, B, form, 1.5, -0.5, C0, name)
            assert guard, f"{name}: wrote outside C"
        except AssertionError as e:
            fails.append(str(e))
    assert not fails, "\n".join(fails[:10])


def test_split_forms_error_against_true_product(split_loaded):
    # alpha = 1, beta = 0: the error against the exact product is the form's
    # truncation plus FP32 accumulation.
    M, N, K = 96, 160, 640
    A = datagen.lognormal((41, 0), M, K)
    B = datagen.lognormal((41, 1), K, N)
    _, S, T = oracle.ref_gemm(A, B)
    for vid, name, form in split_loaded:
        C, _ = run_gemm(vid, A, B, np.full((M, N), np.nan, np.float32), 1.0, 0.0)
        n = len(pr.PAIRS[form])
        bound = (pr.truncation_bound(form) + 4.2 * n * K * 2.0 ** -24) * T
        assert np.all(np.abs(C - S) <= bound), name


def test_bf16_forms_exact_on_bf16_values(split_loaded):
    # Small integers are bf16 values: the bf16 forms are exact when the
    # partial sums stay below 2^24.  The scaled FP16 forms are left out:
    # |x| <= 100 scales by 2^8, so their products reach 2^30 and the FP32
    # partial sums round.
    M, N, K = 64, 96, 200
    A = datagen.integers((42, 0), M, K, -100, 100)
    B = datagen.integers((42, 1), K, N, -100, 100)
    _, S, _ = oracle.ref_gemm(A, B)
    for vid, name, form in split_loaded:
        if form in SCALED:
            continue
        C, _ = run_gemm(vid, A, B, None, 1.0, 0.0)
        assert np.array_equal(C.astype(np.float64), S), name


def test_fp16_scale_follows_the_data(split_loaded):
    # Scaling the inputs by powers of two changes the prescale but not the
    # result beyond the same power of two.
    M, N, K = 48, 64, 96
    A = datagen.lognormal((43, 0), M, K)
    B = datagen.lognormal((43, 1), K, N)
    for vid, name, form in split_loaded:
        if form not in SCALED:
            continue
        C1, _ = run_gemm(vid, A, B, None, 1.0, 0.0)
        C2, _ = run_gemm(vid, A * np.float32(2.0 ** 20), B * np.float32(2.0 ** -30), None, 1.0, 0.0)
        assert np.array_equal(C1 * np.float32(2.0 ** -10), C2), name


@pytest.mark.parametrize("shape,lds", [((5, 4100, 2500), (0, 0, 0)), ((2100, 3, 7), (1, 1, 1)),
                                       ((300, 300, 300), (3, 5, 2))])
def test_fp16_scale_finds_the_largest_entry(split_loaded, shape, lds):
    # The largest |A| and |B| entries sit in the last row unit and last
    # column of each matrix (long rows span several units of the block-maxima
    # pass).  A scale taken from a smaller maximum would push them past the
    # FP16 range and the result to infinity.
    M, N, K = shape
    A = datagen.lognormal((44, M, N, K, 0), M, K)
    B = datagen.lognormal((44, M, N, K, 1), K, N)
    A[M - 1, K - 1] = np.float32(1e4) * np.max(np.abs(A))
    B[K - 1, N - 1] = np.float32(-1e4) * np.max(np.abs(B))
    ref = {}
    for form in SCALED:
        Cs, Ts = pr.split_form_gemm(A, B, form, 1.0, 0.0, None)
        ref[form] = (Cs, pr.accumulation_tolerance(K, form, 1.0, 0.0, Ts, Cs, None))
    fails = []
    for vid, name, form in split_loaded:
        if form not in SCALED:
            continue
        Cs, tol = ref[form]
        C, guard = run_gemm(vid, A, B, None, 1.0, 0.0, K + lds[0], N + lds[1], N + lds[2])
        bad = ~(np.abs(C.astype(np.float64) - Cs) <= tol)
        if bad.any() or not guard:
            fails.append(f"{name}: {int(bad.sum())} elements off, guard {guard}")
    assert not fails, "\n".join(fails[:10])


def test_fp16_scale_max_at_every_lane_position(split_loaded):
    # The block maxima reduce across the lanes of each wave and across the
    # waves of a block: put the one large entry of A (then of B) at columns
    # that land in each row of 16 lanes, each wave, and the second stride.
    vid, name, _ = next(x for x in split_loaded if x[2] == "fp16s")
    M, N, K = 4, 40, 300
    for col in (0, 5, 15, 16, 31, 32, 47, 48, 63, 64, 130, 200, 255, 256, 299):
        for which in ("A", "B"):
            A = datagen.lognormal((45, col, 0), M, K)
            B = datagen.lognormal((45, col, 1), K, N)
            if which == "A":
                A[M - 1, col] = np.float32(3e4) * np.max(np.abs(A))
            else:
                B[K - 1, col % N] = np.float32(3e4) * np.max(np.abs(B))
            C, _ = run_gemm(vid, A, B, None, 1.0, 0.0)
            _check_form(C, A, B, "fp16s", label=f"{name} large {which} entry at column {col}")


@pytest.mark.parametrize("ea,eb", [(-62, -62), (-100, 100), (60, -60)])
def test_scaled_forms_extreme_magnitudes(split_loaded, ea, eb):
    # Operands far from 1 (uniform entries times 2^ea and 2^eb, exact in
    # FP32): the scale exponents reach 77 + 77 (an unscale factor of 2^-154,
    # below FP32's range as one number, while every element of C is a normal
    # FP32: the tiny operands are taken positive, so no element cancels) and
    # 115 (beyond 100), and every scaled variant must still give the oracle's
    # form value, whose exponent rule has no clamp.
    M, N, K = 72, 136, 264
    A = datagen.uniform((42, ea + 200, 0), M, K) * np.float32(2.0 ** ea)
    B = datagen.uniform((42, eb + 200, 1), K, N) * np.float32(2.0 ** eb)
    if ea < 0 and eb < 0:
        A, B = np.abs(A), np.abs(B)
    fails = []
    for vid, name, form in split_loaded:
        if form not in SCALED:
            continue
        C, guard = run_gemm(vid, A, B, np.full((M, N), np.nan, np.float32), 1.0, 0.0)
        try:
            assert np.isfinite(C).all() and np.any(C != 0), f"{name}: zero or non-finite result"
            _check_form(C, A, B, form, label=name)
            assert guard, f"{name}: wrote outside C"
        except AssertionError as e:
            fails.append(str(e))
    assert not fails, "\n".join(fails[:10])


def test_scaled_forms_zero_operand(split_loaded):
    # An all-zero A: the scale exponent is 0 for it (nothing to scale) and
    # every scaled-form variant writes exact zeros (beta = 0, C poisoned
    # with NaN beforehand).
    M, N, K = 40, 72, 96
    A = np.zeros((M, K), np.float32)
    B = datagen.lognormal((46, 1), K, N)
    for vid, name, form in split_loaded:
        if form not in SCALED:
            continue
        C, guard = run_gemm(vid, A, B, np.full((M, N), np.nan, np.float32), 1.0, 0.0)
        assert guard and np.array_equal(C, np.zeros((M, N), np.float32)), name


def test_presplit_workspace_limit(split_loaded):
    # A pre-split call whose pieces exceed the 1 GiB pieces workspace is
    # refused before any launch: bf16x6 keeps 3 pieces per value, and
    # 2 B * 3 * (Mp + Np) * Kp = 1.6e9 bytes for 16384 x 16384 x 8192.
    vid = next(v for v, name, form in split_loaded if form == "bf16x6" and name.endswith("_l2"))
    M = N = 16384
    K = 8192
    A = torch.empty(M, K, device="cuda")
    B = torch.empty(K, N, device="cuda")
    C = torch.full((M, N), 7.0, device="cuda")   # full size; never written: the call fails first
    rc = abi.lib().sgemm_variant(vid, M, N, K, 1.0, A.data_ptr(), K, B.data_ptr(), N, 0.0,
                                 C.data_ptr(), N, None)
    assert rc == abi.FF_ERR_TOO_LARGE, (rc, abi.last_error())
    assert "pieces" in abi.last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(C == 7.0))

