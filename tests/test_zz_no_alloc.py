"""GPU: the allocation-free entry point sgemm_form_noalloc against the entry
point it mirrors, sgemm_form, and against the oracle.

Each case loads a set and calls sgemm_form_noalloc twice in a row, the
second call on a smaller problem, so that what the first call left in the
fixed scratch array cannot stand in for what the second must compute.  Each
result must equal sgemm_form's on the same inputs bit for bit (same
variant, split count and kernels) and meet the oracle's bound (the FP32
GEMM bound, or the form value's accumulation bound for the 16-bit forms).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import precision_ref as pr
from paper_2507_15277_amd import abi, datagen, tuned

pytestmark = pytest.mark.gpu

FORMS = {"fp32": 0, "bf16x3": 1, "bf16x6": 2, "fp16s": 3, "fp16x3": 4}


def _manifest():
    out = {}
    for line in open(os.path.join(tuned.VARIANT_DIR, "manifest.txt")):
        if not line.startswith("#"):
            out[line.split()[1]] = line.strip()
    return out


def _one_member_set(tmp_path, name, form):
    """A set file whose only member is variant `name`: every shape runs it."""
    desc = _manifest()[name]
    vid = int(desc.split()[0])
    path = tmp_path / f"one_{name}.txt"
    path.write_text(f"fewfit-set 1\narch gfx950\ncodedir {tuned.VARIANT_DIR}\nform {form}\n"
                    f"variant {desc}\nrule 256 256 256 {vid} 0\nend\n")
    return str(path)


def _operands(seed, M, N, K, form):
    if form == "fp32":
        A, B, C0 = datagen.gemm_operands(seed, M, N, K, beta=0.5)
    else:
        A = datagen.lognormal((seed, M, N, K, 0), M, K)
        B = datagen.lognormal((seed, M, N, K, 1), K, N)
        C0 = datagen.uniform((seed, M, N, K, 2), M, N)
    return A, B, C0


def _run(entry, fid, A, B, C0, alpha=1.25, beta=0.5):
    M, K = A.shape
    N = B.shape[1]
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.from_numpy(C0).cuda()
    entry(fid, M, N, K, alpha, dA, K, dB, N, beta, dC, N)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def _check_oracle(C, A, B, C0, form, alpha=1.25, beta=0.5):
    K = A.shape[1]
    if form == "fp32":
        Cref, S, T = oracle.ref_gemm(A, B, alpha, beta, C0)
        tol = oracle.gemm_tolerance(K, alpha, beta, S, T, C0)
    else:
        Cref, Ts = pr.split_form_gemm(A, B, form, alpha, beta, C0)
        tol = pr.accumulation_tolerance(K, form, alpha, beta, Ts, Cref, C0)
    err = np.abs(C.astype(np.float64) - Cref)
    assert (err <= tol).all(), float(np.max(err / np.maximum(tol, 1e-300)))


def _two_calls(fid, form, shapes, seed):
    for i, (M, N, K) in enumerate(shapes):
        A, B, C0 = _operands(seed + i, M, N, K, form)
        want = _run(abi.sgemm_form, fid, A, B, C0)
        got = _run(abi.sgemm_form_noalloc, fid, A, B, C0)
        assert np.array_equal(got, want), (form, (M, N, K), "differs from sgemm_form")
        _check_oracle(got, A, B, C0, form)


# One-member sets, so that the scratch users are certain: K-split slices
# (FP32), FP16 exponents + pieces + slices (fp16s pre-split, split K),
# three-piece planes + slices (bf16x6 pre-split).  Shapes: (first, second).
SCRATCH_CASES = [
    ("sgemm_m32n32k32_i32_w1x1_s4_v4_l1_p16", "fp32", [(200, 136, 3000), (72, 40, 700)]),
    ("sgemmx_fp16s_m64n64k64_i32_w2x2_p8_l2", "fp16s", [(300, 260, 2000), (130, 70, 900)]),
    ("sgemmx_bf16x6_m128n128k32_i32_w2x2_p4_l2", "bf16x6", [(1000, 900, 1500), (200, 100, 600)]),
]


@pytest.mark.parametrize("name,form,shapes", SCRATCH_CASES, ids=[c[0] for c in SCRATCH_CASES])
def test_noalloc_matches_sgemm_form(tmp_path, name, form, shapes):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fid = FORMS[form]
    assert abi.variant_set_load(_one_member_set(tmp_path, name, form)) == 1
    vid = int(_manifest()[name].split()[0])
    M, N, K = shapes[0]
    assert abi.variant_work_groups(vid, M, N, K) > -(-M // int(_manifest()[name].split()[2])) * \
        -(-N // int(_manifest()[name].split()[3])), "the first call must split K over work-groups"
    _two_calls(fid, form, shapes, 70)


@pytest.mark.parametrize("form", list(FORMS))
def test_noalloc_through_committed_sets(form):
    # The k = 4 set of each form, as a user would load it: a mid shape, then
    # a smaller one with long K (split over work-groups in the 16-bit sets).
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fid = FORMS[form]
    assert abi.variant_set_load(tuned.set_path(4, form)) == 4
    _two_calls(fid, form, [(1024, 1024, 1024), (256, 256, 4096)], 80)


def test_noalloc_through_the_mixed_set():
    # The mixed set (members of several forms): one shape its rule sends to
    # an fp16x3 member, then one it sends to an FP32 member, each to its
    # member form's oracle and bitwise equal to sgemm_form.
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert abi.variant_set_load(tuned.set_path(4, "mixed")) == 4
    seen = []
    for i, (M, N, K) in enumerate([(1024, 4096, 256), (256, 256, 4096)]):
        vid = abi.variant_select_form(abi.FF_FORM_MIXED, M, N, K)
        form = abi.FORM_NAMES[int(abi.variant_info(vid).split()[13])]
        seen.append(form)
        A, B, C0 = _operands(90 + i, M, N, K, form)
        want = _run(abi.sgemm_form, abi.FF_FORM_MIXED, A, B, C0)
        got = _run(abi.sgemm_form_noalloc, abi.FF_FORM_MIXED, A, B, C0)
        assert np.array_equal(got, want), ((M, N, K), form, "differs from sgemm_form")
        _check_oracle(got, A, B, C0, form)
    assert seen == ["fp16x3", "fp32"], seen


def test_noalloc_rejects_beyond_the_array(tmp_path):
    # bf16x6 pieces of 8192 x 8192 x 4096 take 2 * 3 * 16384 * 4096 bytes
    # (384 MiB), beyond the 256 MiB array: refused before any launch, C
    # untouched; the allocating entry point (1 GiB pieces workspace) runs it.
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert abi.variant_set_load(_one_member_set(tmp_path, "sgemmx_bf16x6_m128n128k32_i32_w2x2_p4_l2", "bf16x6")) == 1
    M = N = 8192
    K = 4096
    A = torch.zeros(M, K, device="cuda")
    B = torch.zeros(K, N, device="cuda")
    C = torch.full((M, N), 7.0, device="cuda")
    rc = abi.lib().sgemm_form_noalloc(2, M, N, K, 1.0, A.data_ptr(), K, B.data_ptr(), N, 0.0, C.data_ptr(), N,
                                      None)
    assert rc == abi.FF_ERR_TOO_LARGE, (rc, abi.last_error())
    assert "scratch" in abi.last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(C == 7.0))
    abi.sgemm_form(2, M, N, K, 1.0, A, K, B, N, 0.0, C, N)
    torch.cuda.synchronize()
    assert bool(torch.all(C == 0.0))
