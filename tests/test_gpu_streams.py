"""GPU: calls that share the library's per-device buffers (K-split slices,
FP16 exponents, pre-split pieces) issued concurrently on two streams of the
same priority, with no host synchronisation between them.  The library
orders such calls across streams, so every result must equal the result of
the same call made alone (bit for bit) and meet the oracle's bound."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import precision_ref as pr
from paper_2507_15277_amd import abi, datagen, tuned

pytestmark = pytest.mark.gpu


def _vid(name):
    for line in open(os.path.join(tuned.VARIANT_DIR, "manifest.txt")):
        if not line.startswith("#") and line.split()[1] == name:
            return int(line.split()[0])
    raise KeyError(name)


def _problem(seed, M, N, K, lognormal):
    if lognormal:
        A = datagen.lognormal((seed, M, N, K, 0), M, K)
        B = datagen.lognormal((seed, M, N, K, 1), K, N)
    else:
        A, B, _ = datagen.gemm_operands(seed, M, N, K)
    return A, B


def test_two_streams_k_split_and_presplit_variants():
    # Stream 1: an FP32 member that splits K over 16 work-groups (slices in
    # the shared workspace).  Stream 2: an fp16s pre-split member that splits
    # K over 8 (exponents, pieces and slices in the shared buffers).  Four
    # rounds each on different operands, all enqueued before any sync.
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.variant_manifest_load(tuned.VARIANT_DIR)
    jobs = [(_vid("sgemm_m32n32k32_i32_w1x1_s4_v4_l1_p16"), None, (200, 136, 3000)),
            (_vid("sgemmx_fp16s_m64n64k64_i32_w2x2_p8_l2"), "fp16s", (300, 260, 2000))]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    problems = []
    for r in range(4):
        for j, (vid, form, (M, N, K)) in enumerate(jobs):
            A, B = _problem(90 + 10 * r + j, M, N, K, form is not None)
            dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            problems.append((j, vid, form, A, B, dA, dB, torch.full((M, N), float("nan"), device="cuda")))
    torch.cuda.synchronize()
    for j, vid, form, A, B, dA, dB, dC in problems:                  # concurrent
        M, K = A.shape
        N = B.shape[1]
        abi.sgemm_variant(vid, M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N, streams[j])
    torch.cuda.synchronize()
    for j, vid, form, A, B, dA, dB, dC in problems:
        M, K = A.shape
        N = B.shape[1]
        alone = torch.full((M, N), float("nan"), device="cuda")
        abi.sgemm_variant(vid, M, N, K, 1.0, dA, K, dB, N, 0.0, alone, N)
        torch.cuda.synchronize()
        assert torch.equal(dC, alone), (vid, "concurrent result differs from the call made alone")
        C = dC.cpu().numpy().astype(np.float64)
        if form is None:
            Cref, S, T = oracle.ref_gemm(A, B)
            tol = oracle.gemm_tolerance(K, 1.0, 0.0, S, T)
        else:
            Cref, Ts = pr.split_form_gemm(A, B, form)
            tol = pr.accumulation_tolerance(K, form, 1.0, 0.0, Ts, Cref)
        assert (np.abs(C - Cref) <= tol).all(), vid


@pytest.mark.parametrize("form", ["fp16x3", "bf16x6"])
def test_two_streams_through_the_form_set(form):
    # sgemm_form through the committed k = 4 set on two streams at once:
    # 2048^3 runs a pre-split member (pieces), 256 x 256 x 4096 a K-split one.
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fid = pr.FORMS[form]
    assert abi.variant_set_load(tuned.set_path(4, form)) == 4
    shapes = [(2048, 2048, 2048), (256, 256, 4096), (2048, 2048, 2048), (256, 256, 4096)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    calls = []
    for i, (M, N, K) in enumerate(shapes):
        A, B = _problem(120 + i, M, N, K, True)
        calls.append((i, A, B, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(),
                      torch.full((M, N), float("nan"), device="cuda")))
    torch.cuda.synchronize()
    for i, A, B, dA, dB, dC in calls:
        M, K = A.shape
        N = B.shape[1]
        abi.sgemm_form(fid, M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N, streams[i % 2])
    torch.cuda.synchronize()
    for i, A, B, dA, dB, dC in calls:
        M, K = A.shape
        N = B.shape[1]
        alone = torch.full((M, N), float("nan"), device="cuda")
        abi.sgemm_form(fid, M, N, K, 1.0, dA, K, dB, N, 0.0, alone, N)
        torch.cuda.synchronize()
        assert torch.equal(dC, alone), (form, (M, N, K), "concurrent result differs from the call made alone")
        rng = np.random.default_rng([130, i])
        rows = np.unique(np.r_[0, M - 1, rng.integers(0, M, 12)])
        cols = np.unique(np.r_[0, N - 1, rng.integers(0, N, 12)])
        # The form's pieces over the whole matrices (the FP16 scale is per
        # matrix), then their kept products on the sampled rows and columns.
        pa, ea = pr.pieces(A, form)
        pb, eb = pr.pieces(B, form)
        Cs = np.zeros((len(rows), len(cols)))
        Ts = np.zeros_like(Cs)
        for ta, tb in pr.PAIRS[form]:
            _, sv, tv = oracle.ref_gemm(np.ascontiguousarray(pa[ta][rows]), np.ascontiguousarray(pb[tb][:, cols]))
            Cs += sv
            Ts += tv
        sc = 2.0 ** -(ea + eb)
        tol = pr.accumulation_tolerance(K, form, 1.0, 0.0, sc * Ts)
        got = dC.cpu().numpy()[np.ix_(rows, cols)].astype(np.float64)
        assert (np.abs(got - sc * Cs) <= tol).all(), (form, (M, N, K))
