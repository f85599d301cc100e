"""GPU: the runtime's set dispatch (variant_set_load + variant_select) against
the oracle's rule on the committed set files, and sgemm() through a set
against the FP64 oracle.

The runtime tabulates the wave correction from the device it runs on; the
oracle is given the same inputs: the set file's training shapes and member
log-slowdowns, work-group counts of each member's launch (tiles times K
splits) as the runtime itself reports them (``variant_work_groups``), and
the device's compute-unit count.  Those counts are checked against
hand-worked values here and against ``space.Variant.work_groups``, whose
own hand-worked cases run on the CPU.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import ptune_ref as pr
from paper_2507_15277_amd import abi, datagen, space, tuned
from tests.gpu_util import run_gemm

pytestmark = pytest.mark.gpu

SETS_DIR = os.path.dirname(tuned.set_path(4))
FORMS = {"fp32": 0, "bf16x3": 1, "bf16x6": 2, "fp16s": 3, "fp16x3": 4, "mixed": 5}


def _parse(path):
    """(form, [member ids], {id: Variant}, [training shapes], cost rows)."""
    form, members, variants, train, cost = 0, [], {}, [], []
    for line in open(path):
        f = line.split("#")[0].split()
        if not f:
            continue
        if f[0] == "form":
            form = FORMS[f[1]]
        elif f[0] == "variant":
            vid = int(f[1])
            members.append(vid)
            variants[vid] = space.Variant(*[int(x) for x in f[3:]])
        elif f[0] == "rule":
            train.append(tuple(int(x) for x in f[1:4]))
            cost.append([float(x) for x in f[5:]])
    return form, members, variants, train, cost


def _queries():
    rng = np.random.default_rng(31)
    q = list(datagen.grid27()) + list(datagen.square_shapes()) + list(datagen.SKEWED_EXTRA)
    q += [(1, 1, 1), (0, 64, 64), (64, 0, 64), (64, 64, 0), (17, 4099, 255), (4097, 33, 1025)]
    q += [tuple(int(x) for x in 2 ** rng.uniform(4, 13, 3)) for _ in range(40)]
    return q


@pytest.fixture(scope="module")
def cus():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.cuda.get_device_properties(0).multi_processor_count


@pytest.mark.parametrize("fname", sorted(f for f in os.listdir(SETS_DIR) if f.endswith(".txt")))
def test_select_matches_oracle_rule(cus, fname):
    path = os.path.join(SETS_DIR, fname)
    form, members, variants, train, cost = _parse(path)
    assert abi.variant_set_load(path) == len(members)
    gt = [[abi.variant_work_groups(v, *s) for v in members] for s in train]
    assert gt == [[variants[v].work_groups(*s) for v in members] for s in train], fname
    for q in _queries():
        gq = [abi.variant_work_groups(v, *q) for v in members]
        assert gq == [variants[v].work_groups(*q) for v in members], (fname, q)
        want = pr.dispatch(train, members, cost, *q, gt, gq, cus)
        assert abi.variant_select_form(form, *q) == want, (fname, q)
    # Every training shape gets its own rule winner.
    for s, row in zip(train, cost):
        assert abi.variant_select_form(form, *s) == members[int(np.argmin(row))], (fname, s)


# Hand-worked work-group counts of manifest variants, as the runtime must
# report them: (variant name, shape, count, how it arises).
HAND_GROUPS = [
    ("sgemm_m64n128k32_i16_w2x2_s2_v4_l1_d2", (4096, 4096, 4096), 64 * 32, "64 x 32 tiles"),
    ("sgemm_m64n64k64_i32_w2x2_s2_v4_l1_d2", (300, 500, 700), 5 * 8, "ceil(300/64) x ceil(500/64)"),
    ("sgemm_m32n32k32_i32_w1x1_s4_v4_l1_p4", (256, 256, 4096), 64 * 4, "64 tiles x 4 splits of 32 slabs"),
    ("sgemm_m64n64k64_i32_w2x2_s2_v4_l2_p8", (256, 256, 640), 16 * 5, "10 slabs: 5 non-empty splits of 2"),
    ("sgemm_m128n128k16_i32_w2x2_s1_v4_l1_p4", (4096, 2048, 4096), 32 * 16 * 4, "4 slices of 32 MiB fit"),
    ("sgemm_m128n128k16_i32_w2x2_s1_v4_l1_p4", (8192, 8192, 1024), 64 * 64, "a 256 MiB slice does not fit"),
    ("sgemm_m128n128k16_i32_w2x2_s1_v4_l1_p2", (4096, 4096, 1024), 32 * 32 * 2, "2 slices of 64 MiB fit"),
    ("sgemm_m64n64k16_i32_w2x2_s1_v4_l1_p4", (0, 64, 64), 0, "empty"),
]


def test_runtime_work_groups_hand_cases(cus):
    abi.variant_manifest_load(tuned.VARIANT_DIR)
    for name, shape, want, why in HAND_GROUPS:
        assert abi.variant_work_groups(_variant_id(name), *shape) == want, (name, shape, why)


@pytest.mark.parametrize("shape", [(256, 1024, 1024), (1024, 1024, 1024), (300, 500, 700), (4096, 256, 1024)])
def test_sgemm_through_set(cus, shape):
    M, N, K = shape
    assert abi.variant_set_load(tuned.set_path(4)) == 4
    A, B, _ = datagen.gemm_operands(41, M, N, K)
    C, guard_ok = run_gemm(None, A, B, None, 1.0, 0.0)
    assert guard_ok, shape
    Cref, S, T = oracle.ref_gemm(A, B)
    tol = oracle.gemm_tolerance(K, 1.0, 0.0, S, T, None)
    assert np.all(np.abs(C.astype(np.float64) - Cref) <= tol), shape


def _variant_id(name):
    for line in open(os.path.join(tuned.VARIANT_DIR, "manifest.txt")):
        f = line.split()
        if not line.startswith("#") and f[1] == name:
            return int(f[0])
    raise KeyError(name)


def test_dispatch_path_graph_replays(cus):
    # The calls a user would capture: a K-split FP32 variant (GEMM, then the
    # fixed-order reduction) and a pre-split form (two split passes, GEMM,
    # reduction), captured once and replayed three times with eager work in
    # between.  Every replay must reproduce the eager result bit for bit.
    abi.variant_manifest_load(tuned.VARIANT_DIR)
    fp32_split = next(int(l.split()[0]) for l in open(os.path.join(tuned.VARIANT_DIR, "manifest.txt"))
                      if not l.startswith("#") and int(l.split()[12]) > 1 and int(l.split()[13]) == 0)
    presplit = next(int(l.split()[0]) for l in open(os.path.join(tuned.VARIANT_DIR, "manifest.txt"))
                    if not l.startswith("#") and int(l.split()[13]) == 2 and int(l.split()[10]) == 2
                    and int(l.split()[12]) > 1)
    M, N, K = 192, 160, 1000
    A, B, C0 = datagen.gemm_operands(51, M, N, K, beta=0.5)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C1 = torch.from_numpy(C0).cuda()
    C2 = torch.from_numpy(C0).cuda()
    start1, start2 = C1.clone(), C2.clone()

    def calls(stream):
        abi.sgemm_variant(fp32_split, M, N, K, 1.25, dA, K, dB, N, 0.5, C1, N, stream)
        abi.sgemm_variant(presplit, M, N, K, 1.25, dA, K, dB, N, 0.5, C2, N, stream)

    calls(torch.cuda.current_stream())
    torch.cuda.synchronize()
    eager1, eager2 = C1.clone(), C2.clone()
    Cref, S, T = oracle.ref_gemm(A, B, 1.25, 0.5, C0)
    tol = oracle.gemm_tolerance(K, 1.25, 0.5, S, T, C0)
    assert np.all(np.abs(eager1.cpu().numpy().astype(np.float64) - Cref) <= tol)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    C1.copy_(start1)
    C2.copy_(start2)
    with torch.cuda.stream(side):
        calls(side)                                      # warm the side stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        calls(torch.cuda.current_stream())
    for r in range(3):
        C1.copy_(start1)                                 # eager work between replays
        C2.copy_(start2)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(C1, eager1), f"replay {r}: K-split FP32 result differs"
        assert torch.equal(C2, eager2), f"replay {r}: pre-split result differs"


def test_mixed_set_graph_replays():
    # The accuracy-targeted set as a captured caller would use it: a shape its
    # rule sends to the fp16x3 pre-split member (scale passes, split passes,
    # GEMM) and one it sends to an FP32 member, through sgemm_form and the
    # allocation-free entry point, captured once and replayed three times with
    # eager work in between; every replay reproduces the eager result exactly.
    assert abi.variant_set_load(tuned.set_path(4, "mixed")) == 4
    shapes = [(1024, 4096, 256), (256, 256, 4096)]
    forms = [abi.FORM_NAMES[int(abi.variant_info(abi.variant_select_form(abi.FF_FORM_MIXED, *s)).split()[13])]
             for s in shapes]
    assert forms == ["fp16x3", "fp32"], forms
    ops = []
    for i, (M, N, K) in enumerate(shapes):
        A, B, C0 = datagen.gemm_operands(61 + i, M, N, K, beta=0.5)
        ops.append((M, N, K, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), torch.from_numpy(C0).cuda()))
    outs = [C0.clone() for (_, _, _, _, _, C0) in ops] + [ops[0][5].clone()]

    def calls(stream):
        for (M, N, K, dA, dB, _), C in zip(ops, outs):
            abi.sgemm_form(abi.FF_FORM_MIXED, M, N, K, 1.25, dA, K, dB, N, 0.5, C, N, stream)
        M, N, K, dA, dB, _ = ops[0]
        abi.sgemm_form_noalloc(abi.FF_FORM_MIXED, M, N, K, 1.25, dA, K, dB, N, 0.5, outs[2], N, stream)

    def reset():
        for C, src in zip(outs, [o[5] for o in ops] + [ops[0][5]]):
            C.copy_(src)

    calls(torch.cuda.current_stream())
    torch.cuda.synchronize()
    eager = [C.clone() for C in outs]
    assert torch.equal(eager[2], eager[0]), "the allocation-free call differs from sgemm_form"
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    reset()
    with torch.cuda.stream(side):
        calls(side)                                      # warm the side stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        calls(torch.cuda.current_stream())
    for r in range(3):
        reset()                                          # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for j, (C, E) in enumerate(zip(outs, eager)):
            assert torch.equal(C, E), f"replay {r}: output {j} differs from the eager result"
