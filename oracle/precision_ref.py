"""Reference oracle for the split-precision GEMM forms -- TEST INFRASTRUCTURE ONLY.

The precision forms compute an FP32 GEMM from 16-bit pieces of the FP32
operands with FP32 accumulation:

* bf16x3: x = hi + lo + d, hi = bf16(x), lo = bf16(x - hi); the product keeps
  lo_a hi_b + hi_a lo_b + hi_a hi_b.
* bf16x6: x = hi + mid + lo + d, mid = bf16(x - hi), lo = bf16(x - hi - mid);
  the product keeps the six term products of total order <= 2.
* fp16s: x * 2^e rounded to FP16, e per matrix with max|x| * 2^e in
  [2^14, 2^15); one product, scaled back by 2^-(ea + eb).
* fp16x3: the same scaled value s = x * 2^e in two FP16 pieces,
  hi = fp16(s), lo = fp16(s - hi); the product keeps lo_a hi_b + hi_a lo_b
  + hi_a hi_b, scaled back by 2^-(ea + eb).

Here every piece is formed exactly as defined (round to nearest, ties to
even), each kept term product is summed in FP64 with the plain GEMM oracle
(products of 16-bit values are exact in FP64), and the result is the exact
value the form aims at before FP32 accumulation.  A GPU result of the form
must match it within the FP32 accumulation bound of its term products.
"""
from __future__ import annotations

import math

import numpy as np

from . import ref_gemm, U32

FORMS = {"bf16x3": 1, "bf16x6": 2, "fp16s": 3, "fp16x3": 4}
PAIRS = {
    "bf16x3": [(1, 0), (0, 1), (0, 0)],
    "bf16x6": [(2, 0), (0, 2), (1, 1), (1, 0), (0, 1), (0, 0)],
    "fp16s": [(0, 0)],
    "fp16x3": [(1, 0), (0, 1), (0, 0)],
}
TERMS = {"bf16x3": 2, "bf16x6": 3, "fp16s": 1, "fp16x3": 2}


def bf16_rne(x):
    """Round FP32 values to bfloat16 (8 significant bits), nearest, ties to
    even, returned as FP32.  Finite inputs only."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).reshape(x.shape)


def split_bf16(x, terms):
    """[hi, (mid,) lo] with x = sum(pieces) + residual; residuals exact in FP32."""
    x = np.asarray(x, dtype=np.float32)
    out, r = [], x.copy()
    for _ in range(terms):
        p = bf16_rne(r)
        out.append(p)
        r = (r - p).astype(np.float32)      # exact: fits in FP32
    return out


def fp16_exponent(amax):
    """e with amax * 2^e in [2^14, 2^15) (0 when amax == 0)."""
    if amax == 0.0:
        return 0
    _, E = math.frexp(float(amax))          # amax = f * 2^E, f in [0.5, 1)
    return 15 - E


def split_fp16(x):
    """(x * 2^e rounded to FP16 then widened to FP32, e)."""
    x = np.asarray(x, dtype=np.float32)
    e = fp16_exponent(float(np.max(np.abs(x))) if x.size else 0.0)
    scaled = (x.astype(np.float64) * 2.0 ** e).astype(np.float32)
    return scaled.astype(np.float16).astype(np.float32), e


def split_fp16_pieces(x, terms):
    """([hi, lo, ...], e): s = x * 2^e (e as in split_fp16), hi = fp16(s) and
    each later piece the FP16 rounding of the residual left so far; pieces
    widened to FP32.  The residuals are exact in FP32."""
    x = np.asarray(x, dtype=np.float32)
    e = fp16_exponent(float(np.max(np.abs(x))) if x.size else 0.0)
    r = (x.astype(np.float64) * 2.0 ** e).astype(np.float32)
    out = []
    for _ in range(terms):
        p = r.astype(np.float16).astype(np.float32)
        out.append(p)
        r = (r - p).astype(np.float32)
    return out, e


def pieces(x, form):
    """The 16-bit pieces of an FP32 matrix for `form` (as FP32 arrays) and the
    power-of-two exponent applied (0 for the BF16 forms)."""
    if form == "fp16s":
        p, e = split_fp16(x)
        return [p], e
    if form == "fp16x3":
        return split_fp16_pieces(x, 2)
    return split_bf16(x, TERMS[form]), 0


def split_form_gemm(A, B, form, alpha=1.0, beta=0.0, C0=None):
    """Exact (FP64) value of the form before FP32 accumulation:

    ``Csplit = alpha * 2^-(ea+eb) * sum_pairs A_ta @ B_tb + beta * C0`` and
    ``Tsplit = |alpha| * 2^-(ea+eb) * sum_pairs |A_ta| @ |B_tb|``.
    """
    pa, ea = pieces(A, form)
    pb, eb = pieces(B, form)
    M, N = A.shape[0], B.shape[1]
    S = np.zeros((M, N))
    T = np.zeros((M, N))
    for ta, tb in PAIRS[form]:
        _, s, t = ref_gemm(np.ascontiguousarray(pa[ta]), np.ascontiguousarray(pb[tb]))
        S += s
        T += t
    sc = 2.0 ** -(ea + eb)
    C = alpha * sc * S
    if beta != 0.0:
        C = C + beta * np.asarray(C0, np.float64)
    return C, abs(alpha) * sc * T


def accumulation_tolerance(K, form, alpha, beta, Tsplit, Csplit=None, C0=None):
    """Bound on |C_gpu - Csplit|: FP32 accumulation of the kept term products
    (4 * n_products * K * u * Tsplit, as for the FP32 GEMM) plus the
    epilogue's roundings when alpha != 1 or beta != 0 (and the unscale of the
    FP16 form is exact)."""
    n = len(PAIRS[form])
    tol = 4.0 * n * K * U32 * np.asarray(Tsplit)
    if alpha != 1.0 or beta != 0.0:
        extra = np.abs(np.asarray(Csplit))
        if beta != 0.0:
            extra = extra + 2.0 * abs(beta) * np.abs(np.asarray(C0, np.float64))
        tol = tol + 2.0 * U32 * extra
    return tol


def truncation_bound(form):
    """Per-product relative error of dropping the residuals and the omitted
    term products, as a multiple of |a||b| (derived from |x - hi| <= 2^-8|x|
    for round-to-nearest bf16 and |x - fp16(x)| <= 2^-11|x| for normal fp16).
    fp16x3: with d = s - hi - lo, |lo| <= 2^-11 |s| and |d| <= 2^-22 |s|
    while the residual s - hi is an FP16 normal or |s| >= 2^-3 (entries
    within 2^18 of the matrix's largest magnitude); the dropped
    hi_a d_b + d_a hi_b + lo_a lo_b + smaller come to 3.01 * 2^-22 |a||b|."""
    if form == "bf16x3":
        return 3.1 * 2.0 ** -16
    if form == "bf16x6":
        return 4.2 * 2.0 ** -24
    if form == "fp16x3":
        return 3.1 * 2.0 ** -22
    return 2.1 * 2.0 ** -11
