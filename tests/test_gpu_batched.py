"""Grouped persistent launches: parity of every problem of a batch with the
FP64 oracle, for the vector and the scalar kernels, and replays of a
captured HIP graph checked against the eager result."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2507_15277_amd import abi, batched, datagen, tuned
from paper_2507_15277_amd.tune import read_manifest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def loaded():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abi.variant_manifest_load(tuned.VARIANT_DIR)
    return [vid for vid, _, prec in read_manifest(with_prec=True) if prec == 0]


def _small_batch(seed, count=40):
    shapes = batched.batch_shapes(count, seed, lo=16, hi=320)
    ops = [(datagen.uniform((60, seed, i, 0), M, K), datagen.uniform((60, seed, i, 1), K, N))
           for i, (M, N, K) in enumerate(shapes)]
    return shapes, ops


def _check_batch(batch, ops, label):
    fails = []
    for i, (A, B) in enumerate(ops):
        C = batch.result(i).cpu().numpy().astype(np.float64)
        _, S, T = oracle.ref_gemm(A, B)
        K = A.shape[1]
        if not np.all(np.abs(C - S) <= 4 * K * 2.0 ** -24 * T):
            fails.append(f"{label}: problem {i} {A.shape[0]}x{B.shape[1]}x{K}")
    return fails


def test_batch_shapes_recipe():
    s = batched.batch_shapes(2000, 0)
    a = np.array(s)
    assert a.shape == (2000, 3) and a.min() >= 16 and a.max() <= 1024 and np.all(a % 16 == 0)
    # log-uniform: the median size is near sqrt(16 * 1024) = 128
    assert 96 <= np.median(a) <= 176


def test_grouped_matches_oracle(loaded):
    shapes, ops = _small_batch(1)
    picks = loaded[:: max(1, len(loaded) // 24)]
    fails = []
    for vid in picks:
        batch = batched.Batch(shapes, host_ops=ops)
        plan = batched.GroupedPlan(batch, list(range(len(shapes))), vid)
        plan.launch()
        torch.cuda.synchronize()
        fails += _check_batch(batch, ops, abi.variant_info(vid).split()[1] + (" vec" if plan.vec else ""))
    assert not fails, fails[:10]


def test_grouped_scalar_kernel_and_padding(loaded):
    # N not a multiple of 4, one problem with N = 3, odd leading dimensions:
    # the register-staged variants of load width 2 take their vector kernel
    # (the load vector that straddles N is moved into place), the others the
    # scalar-load kernel; padding columns hold NaN and must not leak in.
    shapes = [(37, 29, 53), (16, 16, 16), (70, 45, 33), (5, 3, 2)]
    ops, descs = [], []
    buf = []
    for i, (M, N, K) in enumerate(shapes):
        A = datagen.uniform((61, i, 0), M, K, ld=K + 1)
        B = datagen.uniform((61, i, 1), K, N, ld=N + 3)
        ops.append((np.ascontiguousarray(A), np.ascontiguousarray(B)))
        dA = torch.from_numpy(A.base.copy()).cuda()
        dB = torch.from_numpy(B.base.copy()).cuda()
        dC = torch.full((M, N + 2), float("nan"), device="cuda")
        buf.append((dA, dB, dC))
        descs.append((dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), K + 1, N + 3, N + 2, M, N, K, 0))
    for vid in loaded[:: max(1, len(loaded) // 12)]:
        d = np.array(descs, dtype=abi.gemm_desc_dtype())
        total, prefix, vec = abi.sgemm_grouped_plan(vid, d)
        desc = abi.variant_info(vid).split()
        assert bool(vec) == (int(desc[10]) == 1 and 1 < int(desc[9]) <= 3), desc   # LDS mode 1, VW <= min N
        d_dev = torch.from_numpy(d.view(np.uint8)).cuda()
        p_dev = torch.from_numpy(prefix).cuda()
        for (_, _, dC) in buf:
            dC.fill_(float("nan"))
        abi.sgemm_grouped(vid, len(shapes), d_dev, p_dev, total, 1.0, 0.0, vec)
        torch.cuda.synchronize()
        for i, ((A, B), (_, _, dC)) in enumerate(zip(ops, buf)):
            C = dC.cpu().numpy()
            M, N = C.shape[0], shapes[i][1]
            assert np.all(np.isnan(C[:, N:])), "padding written"
            _, S, T = oracle.ref_gemm(A, B)
            assert np.all(np.abs(C[:, :N] - S) <= 4 * A.shape[1] * 2.0 ** -24 * T), (vid, i)


def test_grouped_vector_kernel_unaligned_rows(loaded):
    # N a multiple of 4 in every problem, K and the leading dimensions of A
    # and B odd: the register-staged variants' plans take the vector kernel
    # (4-byte aligned rows, the K tail element by element), the others the
    # scalar one.  NaN in the padding must not leak in.
    shapes = [(37, 28, 53), (16, 16, 17), (70, 44, 33), (5, 4, 2), (130, 96, 131)]
    ops, descs, buf = [], [], []
    for i, (M, N, K) in enumerate(shapes):
        A = datagen.uniform((62, i, 0), M, K, ld=K + 2)
        B = datagen.uniform((62, i, 1), K, N, ld=N + 1)
        ops.append((np.ascontiguousarray(A), np.ascontiguousarray(B)))
        dA = torch.from_numpy(A.base.copy()).cuda()
        dB = torch.from_numpy(B.base.copy()).cuda()
        dC = torch.full((M, N + 2), float("nan"), device="cuda")
        buf.append((dA, dB, dC))
        descs.append((dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), A.base.shape[1], N + 1, N + 2, M, N, K, 0))
    took_vector = 0
    for vid in loaded[:: max(1, len(loaded) // 16)]:
        d = np.array(descs, dtype=abi.gemm_desc_dtype())
        total, prefix, vec = abi.sgemm_grouped_plan(vid, d)
        desc = abi.variant_info(vid).split()
        assert bool(vec) == (int(desc[10]) == 1 and int(desc[9]) > 1), desc   # LDS mode 1, VW > 1
        took_vector += bool(vec)
        d_dev = torch.from_numpy(d.view(np.uint8)).cuda()
        p_dev = torch.from_numpy(prefix).cuda()
        for (_, _, dC) in buf:
            dC.fill_(float("nan"))
        abi.sgemm_grouped(vid, len(shapes), d_dev, p_dev, total, 1.0, 0.0, vec)
        torch.cuda.synchronize()
        for i, ((A, B), (_, _, dC)) in enumerate(zip(ops, buf)):
            C = dC.cpu().numpy()
            N = shapes[i][1]
            assert np.all(np.isnan(C[:, N:])), "padding written"
            _, S, T = oracle.ref_gemm(A, B)
            assert np.all(np.abs(C[:, :N] - S) <= 4 * A.shape[1] * 2.0 ** -24 * T), (vid, i)
    assert took_vector > 0


def test_grouped_graph_replays(loaded):
    shapes, ops = _small_batch(2, count=30)
    batch = batched.Batch(shapes, host_ops=ops)
    idx = list(range(len(shapes)))
    halves = [idx[::2], idx[1::2]]
    plans = [batched.GroupedPlan(batch, h, loaded[(7 * j) % len(loaded)]) for j, h in enumerate(halves)]
    for p in plans:
        p.launch()
    torch.cuda.synchronize()
    eager = batch.C.clone()
    assert not _check_batch(batch, ops, "eager")
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for p in plans:
            p.launch(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        for p in plans:
            p.launch(stream=torch.cuda.current_stream())
    for r in range(3):
        batch.C.zero_()                  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.C, eager), f"replay {r} differs from the eager result"


def test_concurrent_launches_and_graph_replays(loaded):
    # Three plans of disjoint problems on three streams (forked from and
    # joined back into the current stream), eagerly and captured in a graph
    # replayed three times with eager work between: each result against the
    # oracle and every replay against the eager result.
    shapes, ops = _small_batch(3, count=36)
    batch = batched.Batch(shapes, host_ops=ops)
    idx = list(range(len(shapes)))
    thirds = [idx[0::3], idx[1::3], idx[2::3]]
    plans = [batched.GroupedPlan(batch, t, loaded[(11 * j + 3) % len(loaded)]) for j, t in enumerate(thirds)]
    sides = [torch.cuda.Stream() for _ in plans[1:]]
    main = torch.cuda.current_stream()
    batch.C.zero_()
    batched.launch_concurrent(plans, main, sides)
    torch.cuda.synchronize()
    assert not _check_batch(batch, ops, "concurrent")
    eager = batch.C.clone()
    warm = torch.cuda.Stream()
    warm.wait_stream(main)
    with torch.cuda.stream(warm):
        batched.launch_concurrent(plans, warm, sides)
    main.wait_stream(warm)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batched.launch_concurrent(plans, torch.cuda.current_stream(), sides)
    for r in range(3):
        batch.C.zero_()                  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.C, eager), f"replay {r} differs from the eager result"


def test_plan_rejects_bad_problems(loaded):
    d = np.zeros(2, dtype=abi.gemm_desc_dtype())
    d[0] = (16, 16, 16, 4, 4, 4, 4, 4, 4, 0)
    d[1] = (16, 16, 16, 3, 4, 4, 4, 4, 4, 0)     # lda < K
    with pytest.raises(abi.FewfitError):
        abi.sgemm_grouped_plan(loaded[0], d)


def _committed_bucket_variants():
    """(count, bucket variant ids, size buckets before any K cut, whether the
    largest was cut at its median K) of the committed batched run."""
    import json
    rep = json.load(open(os.path.join(os.path.dirname(tuned.VARIANT_DIR), "data", "mi355x_batched.json")))
    names = [rep["bucket_variants"][str(b)]["name"] for b in range(rep["buckets"])]
    ids = {l.split()[1]: int(l.split()[0]) for l in open(os.path.join(tuned.VARIANT_DIR, "manifest.txt"))
           if not l.startswith("#")}
    split_k = bool(rep.get("split_k", False))
    return rep["count"], [ids[n] for n in names], rep["buckets"] - int(split_k), split_k


def test_full_batch_2000_against_oracle(loaded):
    # The batched workload at full size: 2,000 problems with M, N, K
    # log-uniform on [16, 1024] (multiples of 16), host operands from the
    # seeded generator, one grouped launch per size bucket with the committed
    # bucket variants, then the same launches replayed from a HIP graph.
    # Every problem is checked against the oracle on sampled rows and
    # columns, and over its whole result through C x against A (B x).
    count, bucket_vids, nb, split_k = _committed_bucket_variants()
    assert count == 2000
    shapes = batched.batch_shapes(count, 0)
    ops = [(datagen.uniform((62, i, 0), M, K), datagen.uniform((62, i, 1), K, N))
           for i, (M, N, K) in enumerate(shapes)]
    batch = batched.Batch(shapes, host_ops=ops)
    bucket_of = batched.buckets_of(shapes, nb, split_k)
    assert int(bucket_of.max()) + 1 == len(bucket_vids)
    plans = [batched.GroupedPlan(batch, batched.bucket_members(shapes, bucket_of, b), vid)
             for b, vid in enumerate(bucket_vids)]
    assert sum(p.count for p in plans) == count
    # The largest bucket's tiles outnumber its resident work-groups, so each
    # work-group walks several tiles of the persistent loop.
    assert plans[-1].total > 2 * torch.cuda.get_device_properties(0).multi_processor_count
    batch.C.fill_(float("nan"))
    for p in plans:
        p.launch()
    torch.cuda.synchronize()
    eager = batch.C.clone()

    rng = np.random.default_rng([63])
    fails = []
    U = 2.0 ** -24
    for i, (A, B) in enumerate(ops):
        M, K = A.shape
        N = B.shape[1]
        C = eager[batch.off["C"][i]:batch.off["C"][i] + M * N].view(M, N).cpu().numpy()
        if not np.isfinite(C).all():
            fails.append(f"problem {i} {M}x{N}x{K}: non-finite")
            continue
        rows = np.unique(np.r_[0, M - 1, rng.integers(0, M, 6)])
        cols = np.unique(np.r_[0, N - 1, rng.integers(0, N, 6)])
        _, S, T = oracle.ref_gemm(np.ascontiguousarray(A[rows]), np.ascontiguousarray(B[:, cols]))
        if not np.all(np.abs(C[np.ix_(rows, cols)] - S) <= 4 * K * U * T):
            fails.append(f"problem {i} {M}x{N}x{K}: sampled entries")
        x = rng.uniform(-1.0, 1.0, N)
        A64, B64 = A.astype(np.float64), B.astype(np.float64)
        lhs = np.abs(C.astype(np.float64) @ x - A64 @ (B64 @ x))
        if not np.all(lhs <= 4 * K * U * (np.abs(A64) @ (np.abs(B64) @ np.abs(x)))):
            fails.append(f"problem {i} {M}x{N}x{K}: C x")
    assert not fails, fails[:10]

    # One capture of the four launches, replayed after the result is cleared:
    # bit-equal to the eager launches.
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for p in plans:
            p.launch(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for p in plans:
            p.launch(stream=torch.cuda.current_stream())
    for r in range(2):
        batch.C.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.C, eager), f"graph replay {r} differs from the eager launches"
