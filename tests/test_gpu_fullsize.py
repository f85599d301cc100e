"""GPU parity at the benchmark's full sizes, in the benchmark's launch
configuration: every shape of the {256, 1024, 4096}^3 grid (and the two
skewed shapes off it) through sgemm() dispatched over the k = 4 set, on the
benchmark's seeded inputs.

Two checks per shape:
* sampled outputs: a block of rows x columns (random, plus the first and
  last row and column) against the FP64 oracle on those rows and columns,
  to the elementwise bound 4*K*2^-24*(|A||B|)_ij;
* a property of the whole result: for a random vector x,
  |C x - A (B x)|_i <= 4*K*2^-24 * (|A| (|B| |x|))_i, which the elementwise
  bound implies, computed in FP64 on the host.
The split-precision forms get the same two checks against their exact
form value (pieces formed over the whole matrices, as the kernel forms
them), on the precision workload's lognormal operands.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import precision_ref as pr
from paper_2507_15277_amd import abi, datagen, tuned

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
SHAPES = datagen.grid27() + list(datagen.SKEWED_EXTRA)


def _sample_idx(rng, n, count=24):
    idx = set(rng.choice(n, min(n, count), replace=False).tolist()) | {0, n - 1}
    return np.array(sorted(idx))


def _gpu_gemm(A, B, form=0):
    M, K = A.shape
    N = B.shape[1]
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.full((M, N), float("nan"), device="cuda")
    if form == 0:
        abi.sgemm(M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N)
    else:
        abi.sgemm_form(form, M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


@pytest.fixture(scope="module")
def k4_set():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert abi.variant_set_load(tuned.set_path(4)) == 4


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_fp32_full_size_through_set(k4_set, shape):
    M, N, K = shape
    A, B, _ = datagen.gemm_operands(3, M, N, K)        # the benchmark's inputs
    C = _gpu_gemm(A, B)
    assert np.isfinite(C).all(), shape
    rng = np.random.default_rng([9, M, N, K])
    rows, cols = _sample_idx(rng, M), _sample_idx(rng, N)
    Cref, S, T = oracle.ref_gemm(np.ascontiguousarray(A[rows]), np.ascontiguousarray(B[:, cols]))
    tol = oracle.gemm_tolerance(K, 1.0, 0.0, S, T, None)
    err = np.abs(C[np.ix_(rows, cols)].astype(np.float64) - Cref)
    assert (err <= tol).all(), (shape, float(np.max(err / tol)))
    x = rng.uniform(-1.0, 1.0, N)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    lhs = np.abs(C.astype(np.float64) @ x - A64 @ (B64 @ x))
    bound = 4.0 * K * U * (np.abs(A64) @ (np.abs(B64) @ np.abs(x)))
    assert (lhs <= bound).all(), (shape, float(np.max(lhs / bound)))


@pytest.mark.parametrize("form", ["bf16x3", "bf16x6", "fp16s"])
@pytest.mark.parametrize("shape", [(4096, 4096, 4096), (256, 4096, 1024), (4096, 256, 256), (1024, 1024, 1024)],
                         ids=lambda s: "x".join(map(str, s)))
def test_split_forms_full_size_through_set(form, shape):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fid = pr.FORMS[form]
    assert abi.variant_set_load(tuned.set_path(4, form)) == 4
    M, N, K = shape
    A = datagen.lognormal((50, M, N, K, 0), M, K)
    B = datagen.lognormal((50, M, N, K, 1), K, N)
    C = _gpu_gemm(A, B, fid)
    assert np.isfinite(C).all(), (form, shape)
    # The form's pieces over the whole matrices (the FP16 scale is per matrix).
    pa, ea = pr.pieces(A, form)
    pb, eb = pr.pieces(B, form)
    sc = 2.0 ** -(ea + eb)
    rng = np.random.default_rng([10, M, N, K])
    rows, cols = _sample_idx(rng, M), _sample_idx(rng, N)
    Cs = np.zeros((len(rows), len(cols)))
    Ts = np.zeros_like(Cs)
    for ta, tb in pr.PAIRS[form]:
        _, s, t = oracle.ref_gemm(np.ascontiguousarray(pa[ta][rows]), np.ascontiguousarray(pb[tb][:, cols]))
        Cs += s
        Ts += t
    Cs *= sc
    Ts *= sc
    tol = pr.accumulation_tolerance(K, form, 1.0, 0.0, Ts)
    err = np.abs(C[np.ix_(rows, cols)].astype(np.float64) - Cs)
    assert (err <= tol).all(), (form, shape, float(np.max(err / tol)))
    # Whole result: C x against the form's exact value times x.
    x = rng.uniform(-1.0, 1.0, N)
    exact = np.zeros(M)
    absb = np.zeros(M)
    for ta, tb in pr.PAIRS[form]:
        a64, b64 = pa[ta].astype(np.float64), pb[tb].astype(np.float64)
        exact += a64 @ (b64 @ x)
        absb += np.abs(a64) @ (np.abs(b64) @ np.abs(x))
    lhs = np.abs(C.astype(np.float64) @ x - sc * exact)
    bound = 4.0 * len(pr.PAIRS[form]) * K * U * sc * absb
    assert (lhs <= bound).all(), (form, shape, float(np.max(lhs / bound)))
