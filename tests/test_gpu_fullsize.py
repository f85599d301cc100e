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


@pytest.mark.parametrize("n", datagen.SQUARE_SIZES)
def test_fp32_squares_beta_half_through_set(k4_set, n):
    # The square sweep at beta = 0.5 (C0 uniform on [-1, 1)), through sgemm()
    # and the k = 4 set, on the tuner's seeded inputs: sampled outputs against
    # the oracle, and C x against A (B x) + 0.5 C0 x over the whole result.
    M = N = K = n
    A, B, C0 = datagen.gemm_operands(2, M, N, K, beta=0.5)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.from_numpy(C0).cuda()
    abi.sgemm(M, N, K, 1.0, dA, K, dB, N, 0.5, dC, N)
    torch.cuda.synchronize()
    C = dC.cpu().numpy()
    assert np.isfinite(C).all(), n
    rng = np.random.default_rng([11, n])
    rows, cols = _sample_idx(rng, M), _sample_idx(rng, N)
    C0s = np.ascontiguousarray(C0[np.ix_(rows, cols)])
    Cref, S, T = oracle.ref_gemm(np.ascontiguousarray(A[rows]), np.ascontiguousarray(B[:, cols]), 1.0, 0.5, C0s)
    tol = oracle.gemm_tolerance(K, 1.0, 0.5, S, T, C0s)
    err = np.abs(C[np.ix_(rows, cols)].astype(np.float64) - Cref)
    assert (err <= tol).all(), (n, float(np.max(err / tol)))
    # The elementwise bound summed against |x|; |A B| <= |A||B| covers the
    # epilogue's 2u|alpha A B| term.
    x = rng.uniform(-1.0, 1.0, N)
    A64, B64, C064 = A.astype(np.float64), B.astype(np.float64), C0.astype(np.float64)
    lhs = np.abs(C.astype(np.float64) @ x - (A64 @ (B64 @ x) + 0.5 * (C064 @ x)))
    bound = (4.0 * K + 2.0) * U * (np.abs(A64) @ (np.abs(B64) @ np.abs(x))) + 2.0 * U * 0.5 * (np.abs(C064) @ np.abs(x))
    assert (lhs <= bound).all(), (n, float(np.max(lhs / bound)))


@pytest.mark.parametrize("form", ["bf16x3", "bf16x6", "fp16s", "fp16x3"])
@pytest.mark.parametrize("shape", datagen.grid27(), ids=lambda s: "x".join(map(str, s)))
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


@pytest.mark.parametrize("shape", datagen.grid27(), ids=lambda s: "x".join(map(str, s)))
def test_mixed_set_full_size_meets_target(shape):
    # The mixed set (members of several forms chosen for a normwise error of
    # at most 1e-6 on lognormal operands): each call runs its dispatched
    # member in that member's form, checked to that form's elementwise bound
    # on sampled rows and columns, and the normwise error of 64 sampled rows
    # against the FP64 product must meet the target (the target is on the
    # whole result, which the rows estimate; the 1.25 covers the sampling).
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert abi.variant_set_load(tuned.set_path(4, "mixed")) == 4
    M, N, K = shape
    A = datagen.lognormal((51, M, N, K, 0), M, K)
    B = datagen.lognormal((51, M, N, K, 1), K, N)
    vid = abi.variant_select_form(abi.FF_FORM_MIXED, M, N, K)
    form = abi.FORM_NAMES[int(abi.variant_info(vid).split()[13])]
    C = _gpu_gemm(A, B, abi.FF_FORM_MIXED).astype(np.float64)
    assert np.isfinite(C).all(), shape
    rng = np.random.default_rng([11, M, N, K])
    rows, cols = _sample_idx(rng, M, 64), _sample_idx(rng, N)
    exact_rows, _, _ = oracle.ref_gemm(np.ascontiguousarray(A[rows]), B)
    rel = np.linalg.norm(C[rows] - exact_rows) / np.linalg.norm(exact_rows)
    assert rel <= 1.25e-6, (shape, form, rel)
    if form == "fp32":
        Cref, S, T = oracle.ref_gemm(np.ascontiguousarray(A[rows]), np.ascontiguousarray(B[:, cols]))
        tol = oracle.gemm_tolerance(K, 1.0, 0.0, S, T, None)
        err = np.abs(C[np.ix_(rows, cols)] - Cref)
    else:
        pa, ea = pr.pieces(A, form)
        pb, eb = pr.pieces(B, form)
        sc = 2.0 ** -(ea + eb)
        Cs = np.zeros((len(rows), len(cols)))
        Ts = np.zeros_like(Cs)
        for ta, tb in pr.PAIRS[form]:
            _, s_, t_ = oracle.ref_gemm(np.ascontiguousarray(pa[ta][rows]), np.ascontiguousarray(pb[tb][:, cols]))
            Cs += s_
            Ts += t_
        tol = pr.accumulation_tolerance(K, form, 1.0, 0.0, Ts * sc)
        err = np.abs(C[np.ix_(rows, cols)] - Cs * sc)
    assert (err <= tol).all(), (shape, form, float(np.max(err / tol)))


def test_fp32_output_past_2_31_elements(k4_set):
    # C of 65,543 x 65,543 floats (4.3e9 elements, 17 GB): every row, tile
    # and element offset must be formed in 64 bits.  K = 5, through the set.
    M = N = 65543
    K = 5
    A = datagen.uniform((60, 0), M, K)
    B = datagen.uniform((60, 1), K, N)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.full((M, N), float("nan"), device="cuda")
    abi.sgemm(M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N)
    torch.cuda.synchronize()
    rng = np.random.default_rng([61])
    rows, cols = _sample_idx(rng, M), _sample_idx(rng, N)
    Cref, S, T = oracle.ref_gemm(np.ascontiguousarray(A[rows]), B)
    tol = oracle.gemm_tolerance(K, 1.0, 0.0, S, T, None)
    got = dC[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    assert ((np.abs(got - Cref) <= tol).all()), float(np.max(np.abs(got - Cref) / tol))
    Cref, S, T = oracle.ref_gemm(A, np.ascontiguousarray(B[:, cols]))
    tol = oracle.gemm_tolerance(K, 1.0, 0.0, S, T, None)
    got = dC[:, torch.from_numpy(cols).cuda()].cpu().numpy().astype(np.float64)
    assert ((np.abs(got - Cref) <= tol).all()), float(np.max(np.abs(got - Cref) / tol))
    # The whole result: C x against A (B x) in FP64, 4,096 rows at a time.
    x = rng.uniform(-1.0, 1.0, N)
    dx = torch.from_numpy(x).cuda()
    cx = np.concatenate([(dC[r:r + 4096].double() @ dx).cpu().numpy() for r in range(0, M, 4096)])
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    lhs = np.abs(cx - A64 @ (B64 @ x))
    bound = 4.0 * K * U * (np.abs(A64) @ (np.abs(B64) @ np.abs(x)))
    assert (lhs <= bound).all(), float(np.max(lhs / bound))
    del dC


def _k_past_2_24_operands(M, N, K):
    # A has one 1 every 4,099 columns of a row and B holds integers in
    # [-2, 2] (no short period along k), so every partial sum is an integer
    # below 2^24 and the FP32 result is exact in any summation order:
    # bit-equal to the FP64 oracle.
    k = torch.arange(K, device="cuda")
    dA = (k.unsqueeze(0) % 4099 == torch.arange(M, device="cuda").unsqueeze(1)).float().contiguous()
    kk = (k * 40503 + (k >> 5)).unsqueeze(1)
    dB = ((kk + torch.arange(N, device="cuda").unsqueeze(0) * 3) % 5 - 2).float().contiguous()
    return dA, dB


def test_fp32_k_past_2_24_exact(k4_set):
    # K = 2^24 + 3 (A and B 1 GiB each) through the set, as a user would call
    # it.  The set's rule sends 16 x 16 x K to an unsplit member, one
    # work-group walking all of K.
    M = N = 16
    K = (1 << 24) + 3
    dA, dB = _k_past_2_24_operands(M, N, K)
    dC = torch.full((M, N), float("nan"), device="cuda")
    abi.sgemm(M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N)
    torch.cuda.synchronize()
    Cref, _, _ = oracle.ref_gemm(dA.cpu().numpy(), dB.cpu().numpy())
    assert np.array_equal(dC.cpu().numpy().astype(np.float64), Cref)


@pytest.mark.parametrize("name,splits", [("sgemm_m32n32k32_i32_w1x1_s4_v4_l1_p16", 16),
                                         ("sgemm_m16n16k32_i16_w1x1_s2_v4_l0_p16", 16)])
def test_fp32_k_past_2_24_split_over_work_groups(name, splits):
    # The same exact case through FP32 members that split K over 16
    # work-groups (524,289 slabs of 32: 16 splits of 32,769 slabs), so the
    # partial products and the fixed-order reduction run at K > 2^24.
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.variant_manifest_load(tuned.VARIANT_DIR)
    vid = next(int(l.split()[0]) for l in open(tuned.VARIANT_DIR + "/manifest.txt")
               if not l.startswith("#") and l.split()[1] == name)
    M = N = 16
    K = (1 << 24) + 3
    assert abi.variant_work_groups(vid, M, N, K) == splits   # one tile, 16 splits
    dA, dB = _k_past_2_24_operands(M, N, K)
    dC = torch.full((M, N), float("nan"), device="cuda")
    abi.sgemm_variant(vid, M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N)
    torch.cuda.synchronize()
    Cref, _, _ = oracle.ref_gemm(dA.cpu().numpy(), dB.cpu().numpy())
    assert np.array_equal(dC.cpu().numpy().astype(np.float64), Cref)
