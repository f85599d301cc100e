"""Pins of the split-precision oracle: rounding against library routines,
exactness of the splits, closed forms, and the truncation bounds."""
import numpy as np
import pytest
import torch

import oracle
from oracle import precision_ref as pr
from paper_2507_15277_amd import datagen


def test_bf16_rounding_matches_torch():
    # torch's float32 -> bfloat16 conversion rounds to nearest, ties to even.
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    # Exact ties: lower 16 bits 0x8000, with even and odd upper halves.
    ties = (rng.integers(0x3F000000 >> 16, 0x47000000 >> 16, 2000, dtype=np.uint32) << 16) | 0x8000
    x = np.concatenate([x, ties.view(np.float32), -ties.view(np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(pr.bf16_rne(x), want)


def test_fp16_pieces_match_numpy():
    A = datagen.lognormal((5, 0), 40, 30)
    p, e = pr.split_fp16(A)
    amax = float(np.max(np.abs(A)))
    assert 2.0 ** 14 <= amax * 2.0 ** e < 2.0 ** 15
    assert np.array_equal(p, (A * np.float32(2.0 ** e)).astype(np.float16).astype(np.float32))
    assert pr.fp16_exponent(0.0) == 0
    assert pr.fp16_exponent(1.0) == 14 and pr.fp16_exponent(0.75) == 15


@pytest.mark.parametrize("terms", [2, 3])
def test_bf16_split_is_exact(terms):
    x = datagen.lognormal((6, terms), 1, 5000)[0]
    pieces = pr.split_bf16(x, terms)
    for p in pieces:                      # every piece is a bfloat16 value
        assert np.all((p.view(np.uint32) & 0xFFFF) == 0)
    total = sum(p.astype(np.float64) for p in pieces)
    resid = x.astype(np.float64) - total
    # Each split step leaves at most 2^-8 of the previous residual.
    assert np.all(np.abs(resid) <= 2.0 ** (-8 * terms) * np.abs(x))
    # Closed form: 1 + 2^-10 -> hi = 1, lo = 2^-10.
    hi, lo = pr.split_bf16(np.array([1.0 + 2.0 ** -10], np.float32), 2)
    assert hi[0] == 1.0 and lo[0] == 2.0 ** -10


def test_bf16_forms_exact_on_bf16_inputs():
    # Entries that are already bfloat16 values: lo = 0, so the split forms
    # reproduce the exact product.
    A = datagen.integers((7, 0), 20, 33, -100, 100)
    B = datagen.integers((7, 1), 33, 17, -100, 100)
    _, S, _ = oracle.ref_gemm(A, B)
    for form in ("bf16x3", "bf16x6"):
        C, _ = pr.split_form_gemm(A, B, form)
        assert np.array_equal(C, S)


def test_closed_form_one_plus_eps():
    # A = 1 + 2^-10 (bf16 hi 1, lo 2^-10), B = 1 + 2^-12, K = 1:
    # bf16x3 keeps hi*hi + hi*lo + lo*hi = 1 + 2^-12 + 2^-10, drops 2^-22.
    A = np.array([[1.0 + 2.0 ** -10]], np.float32)
    B = np.array([[1.0 + 2.0 ** -12]], np.float32)
    C, T = pr.split_form_gemm(A, B, "bf16x3")
    assert C[0, 0] == 1.0 + 2.0 ** -12 + 2.0 ** -10
    C6, _ = pr.split_form_gemm(A, B, "bf16x6")
    assert C6[0, 0] == (1.0 + 2.0 ** -10) * (1.0 + 2.0 ** -12)


def test_fp16_two_pieces_match_numpy():
    # hi and lo are numpy's float16 roundings of the scaled value and of the
    # residual; the residual left after lo is within 2^-22 of the scaled
    # value (lognormal entries span 16 binades, inside the 2^18 range).
    A = datagen.lognormal((11, 0), 50, 40)
    (hi, lo), e = pr.split_fp16_pieces(A, 2)
    s = A * np.float32(2.0 ** e)
    assert 2.0 ** 14 <= float(np.max(np.abs(s))) < 2.0 ** 15
    assert np.array_equal(hi, s.astype(np.float16).astype(np.float32))
    assert np.array_equal(lo, (s - hi).astype(np.float16).astype(np.float32))
    d = s.astype(np.float64) - hi - lo
    assert np.all(np.abs(d) <= 2.0 ** -22 * np.abs(s))
    assert np.any(np.abs(d) > 2.0 ** -26 * np.abs(s))     # something is dropped
    # The one-piece split is the fp16s piece.
    (p1,), e1 = pr.split_fp16_pieces(A, 1)
    p, ep = pr.split_fp16(A)
    assert e1 == ep and np.array_equal(p1, p)


def test_fp16x3_closed_form():
    # A = 1 + 2^-12, B = 1 + 2^-13, K = 1: both scale by 2^14; hi = 2^14
    # (the FP16 spacing there is 16), lo = 4 and 2; the form keeps
    # hi*hi + hi*lo + lo*hi = 2^28 + 6 * 2^14 and drops lo*lo = 8, so
    # C = 1 + 2^-12 + 2^-13 (the exact product adds 2^-25).
    A = np.array([[1.0 + 2.0 ** -12]], np.float32)
    B = np.array([[1.0 + 2.0 ** -13]], np.float32)
    (ha, la), ea = pr.split_fp16_pieces(A, 2)
    assert ea == 14 and ha[0, 0] == 2.0 ** 14 and la[0, 0] == 4.0
    C, _ = pr.split_form_gemm(A, B, "fp16x3")
    assert C[0, 0] == 1.0 + 2.0 ** -12 + 2.0 ** -13


def test_fp16x3_exact_on_fp16_inputs():
    # Small integers scale to FP16 values exactly: lo = 0 and the form is
    # the exact product.
    A = datagen.integers((12, 0), 20, 33, -100, 100)
    B = datagen.integers((12, 1), 33, 17, -100, 100)
    _, S, _ = oracle.ref_gemm(A, B)
    C, _ = pr.split_form_gemm(A, B, "fp16x3")
    assert np.array_equal(C, S)


@pytest.mark.parametrize("form", ["bf16x3", "bf16x6", "fp16s", "fp16x3"])
def test_truncation_bound_holds_and_is_not_vacuous(form):
    M, N, K = 24, 20, 300
    A = datagen.lognormal((8, 0), M, K)
    B = datagen.lognormal((8, 1), K, N)
    _, S, T = oracle.ref_gemm(A, B)
    C, _ = pr.split_form_gemm(A, B, form)
    err = np.abs(C - S)
    assert np.all(err <= pr.truncation_bound(form) * T)
    # The form really drops something: the largest error is within a factor
    # 1000 of the bound (a split that kept everything would be exact).
    assert np.max(err / T) > pr.truncation_bound(form) / 1000


def test_alpha_beta_in_split_form():
    M, N, K = 9, 7, 11
    A = datagen.lognormal((9, 0), M, K)
    B = datagen.lognormal((9, 1), K, N)
    C0 = datagen.uniform((9, 2), M, N)
    C, T = pr.split_form_gemm(A, B, "bf16x3", alpha=-0.5, beta=2.0, C0=C0)
    C1, T1 = pr.split_form_gemm(A, B, "bf16x3")
    assert np.allclose(C, -0.5 * C1 + 2.0 * C0.astype(np.float64), rtol=0, atol=1e-12)
    assert np.allclose(T, 0.5 * T1)


def test_lognormal_generator_range():
    x = datagen.lognormal((10, 0), 200, 200)
    a = np.abs(x)
    assert a.min() >= 2.0 ** -8 and a.max() <= 2.0 ** 8
    assert 0.4 < np.mean(x > 0) < 0.6
    # sigma = 2: about 0.56% of the magnitudes fall outside 2^[-8,8].
    frac = np.mean((a == np.float32(2.0 ** -8)) | (a == np.float32(2.0 ** 8)))
    assert 0.002 < frac < 0.01


# ---------------------------------------------------------------------------
# Pins of accumulation_tolerance, the pass bound of every split-form parity
# test: an FP32 accumulation of the kept term products sits inside it, and
# each factor of it (products per k, K, |alpha|, the epilogue term) is needed,
# shown by a legal accumulation or a dropped term that lands between the
# bound and a bound missing that factor.

U = 2.0 ** -24


def _fp32_accumulate(A, B, form, alpha=1.0, beta=0.0, C0=None):
    """FP32 accumulation of the form's kept term products, k by k and pair by
    pair (smallest first, as the kernels issue them), then the exact unscale
    and an FP32 epilogue.  Products of 16-bit pieces are exact in FP32."""
    pa, ea = pr.pieces(A, form)
    pb, eb = pr.pieces(B, form)
    M, K = A.shape
    N = B.shape[1]
    acc = np.zeros((M, N), np.float32)
    for k in range(K):
        for ta, tb in pr.PAIRS[form]:
            prod = np.outer(pa[ta][:, k].astype(np.float64), pb[tb][k, :].astype(np.float64))
            acc = (acc + prod.astype(np.float32)).astype(np.float32)
    v = (acc.astype(np.float64) * 2.0 ** -(ea + eb)).astype(np.float32)
    out = (np.float32(alpha) * v).astype(np.float32)
    if beta != 0.0:
        out = (out + (np.float32(beta) * C0.astype(np.float32)).astype(np.float32)).astype(np.float32)
    return out.astype(np.float64)


@pytest.mark.parametrize("form", ["bf16x3", "bf16x6", "fp16s", "fp16x3"])
@pytest.mark.parametrize("K", [1, 7, 256, 1024])
def test_accumulation_tolerance_holds_for_fp32_accumulation(form, K):
    M, N = 6, 5
    A = datagen.lognormal((13, K), M, K)
    B = datagen.lognormal((14, K), K, N)
    Cs, Ts = pr.split_form_gemm(A, B, form)
    got = _fp32_accumulate(A, B, form)
    tol = pr.accumulation_tolerance(K, form, 1.0, 0.0, Ts, Cs)
    assert np.all(np.abs(got - Cs) <= tol)


# K = 1 constructions: one kept term product (the smallest) is dropped, and
# its size is set between the bound and 1.5x the bound, so the bound must be
# violated; a bound with n^2 products, or without |alpha| in Tsplit, is not.
#   bf16x3: a = 1 + 2^-20 (hi 1, lo 2^-20), b = 1: lo_a hi_b = 16u, bound 12u.
#   bf16x6: a = 1 + 2^-10 + 2^-19 (hi 1, mid 2^-10, lo 2^-19), b = 1:
#           lo_a hi_b = 32u, bound 24u.
#   fp16x3: a = 1 + 2^-20 scales to 2^14 + 2^-6 (hi 2^14, lo 2^-6), b = 1
#           (2^14): lo_a hi_b = 2^8, unscaled by 2^-28 to 16u, bound 12u.
_CALIBRATED = {
    "bf16x3": (1.0 + 2.0 ** -20, (1, 0), 16),
    "bf16x6": (1.0 + 2.0 ** -10 + 2.0 ** -19, (2, 0), 32),
    "fp16x3": (1.0 + 2.0 ** -20, (1, 0), 16),
}


@pytest.mark.parametrize("form", sorted(_CALIBRATED))
@pytest.mark.parametrize("alpha", [1.0, 2.0 ** -40])
def test_accumulation_tolerance_catches_a_dropped_term(form, alpha):
    a, drop, units = _CALIBRATED[form]
    A = np.array([[a]], np.float32)
    B = np.array([[1.0]], np.float32)
    pa, ea = pr.pieces(A, form)
    pb, eb = pr.pieces(B, form)
    dropped = float(pa[drop[0]][0, 0]) * float(pb[drop[1]][0, 0]) * 2.0 ** -(ea + eb)
    assert dropped == units * U
    Cs, Ts = pr.split_form_gemm(A, B, form, alpha=alpha)
    tol = pr.accumulation_tolerance(1, form, alpha, 0.0, Ts, Cs)
    n = len(pr.PAIRS[form])
    assert Ts[0, 0] == pytest.approx(alpha * (1.0 + units * U + 2.0 ** -10 * (form == "bf16x6")), rel=1e-12)
    # The sum with that product dropped is outside the bound, by less than
    # the factor a bound with n^2 products would allow.
    err = abs(alpha) * dropped
    assert err > tol[0, 0]
    assert err < n * tol[0, 0]
    # The kept sum in FP32 is exact here, so inside.
    assert abs(alpha * float(np.float32(1.0 + units * U + 2.0 ** -10 * (form == "bf16x6"))) - Cs[0, 0]) <= tol[0, 0]


def test_accumulation_tolerance_one_piece_form_scales_with_K():
    # fp16s: a = [1, 3 * 2^-22], b = [1, 1] (3 * 2^-22 scales by 2^14 to the
    # FP16 value 3 * 2^-8, exact): dropping the second product loses 12u,
    # above the K = 2 bound of 8u.
    A = np.array([[1.0, 3.0 * 2.0 ** -22]], np.float32)
    B = np.array([[1.0], [1.0]], np.float32)
    Cs, Ts = pr.split_form_gemm(A, B, "fp16s")
    assert Cs[0, 0] == 1.0 + 12 * U
    tol = pr.accumulation_tolerance(2, "fp16s", 1.0, 0.0, Ts, Cs)
    assert 12 * U > tol[0, 0] > 8 * U


def test_accumulation_tolerance_needs_its_K_factor():
    # A legal FP32 order reaches about K u: 1 followed by K - 1 products of
    # 2^-24 (1 + 2^-7), each just above half an ulp of the running sum, so
    # each addition rounds up by nearly half an ulp.  bf16x3 with bf16
    # inputs keeps only hi * hi (lo = 0).
    K = 64
    a = np.full((1, K), 2.0 ** -12 * (1 + 2.0 ** -7), np.float32)
    b = np.full((K, 1), 2.0 ** -12, np.float32)
    a[0, 0] = 1.0
    b[0, 0] = 1.0
    Cs, Ts = pr.split_form_gemm(a, b, "bf16x3")
    got = _fp32_accumulate(a, b, "bf16x3")
    err = abs(got[0, 0] - Cs[0, 0])
    assert err > 0.9 * (K - 1) * U            # close to (K - 1) u
    tol = pr.accumulation_tolerance(K, "bf16x3", 1.0, 0.0, Ts, Cs)
    assert err <= tol[0, 0]
    # A bound without K (4 n u T) would reject this legal result.
    assert err > 4 * 3 * U * Ts[0, 0]


def test_accumulation_tolerance_epilogue_term():
    # A = 0: Tsplit = 0 and the result is beta * C0 rounded in FP32; only the
    # epilogue term admits that rounding.
    M, N, K = 8, 9, 5
    A = np.zeros((M, K), np.float32)
    B = datagen.lognormal((15, 1), K, N)
    C0 = datagen.lognormal((15, 2), M, N)
    beta = float(np.float32(1.0 / 3.0))
    for form in ("bf16x3", "fp16x3"):
        Cs, Ts = pr.split_form_gemm(A, B, form, alpha=1.0, beta=beta, C0=C0)
        assert np.all(Ts == 0.0)
        got = _fp32_accumulate(A, B, form, 1.0, beta, C0)
        err = np.abs(got - Cs)
        assert np.any(err > 0.0)
        tol = pr.accumulation_tolerance(K, form, 1.0, beta, Ts, Cs, C0)
        assert np.all(err <= tol)
    # alpha != 1 alone: the FP32 product alpha * acc rounds once more.
    A = datagen.lognormal((16, 0), M, K)
    alpha = float(np.float32(1.0 / 3.0))
    Cs, Ts = pr.split_form_gemm(A, B, "fp16x3", alpha=alpha)
    got = _fp32_accumulate(A, B, "fp16x3", alpha)
    assert np.all(np.abs(got - Cs) <= pr.accumulation_tolerance(K, "fp16x3", alpha, 0.0, Ts, Cs))
