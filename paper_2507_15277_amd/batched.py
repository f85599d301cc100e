"""Batches of uneven GEMMs: grouped persistent launches, one per size bucket,
captured in a HIP graph.

The batch: ``count`` independent problems with M, N, K each log-uniform on
[16, 1024] and rounded to the nearest multiple of 16.  Problems are split
into size buckets by quantiles of log(M N K); for each bucket the autotuner
times the grouped launch of every FP32 variant and keeps the fastest (the
per-bucket variant).  One batch then costs one grouped launch per bucket,
and the launches are captured once in a HIP graph and replayed.  The
buckets' problems are disjoint, so their launches may also run
concurrently: each on its own stream, forked from and joined back into the
caller's stream (the largest bucket first), eagerly or captured the same
way.  The baseline issues one launch per problem with its bucket's variant.

This is the batched use of the selection machinery: the buckets play the
role of the paper's environments and the total time of the batch is the
single-device form of the fleet objective (Eq. 2).

    python -m paper_2507_15277_amd.batched [--count 2000] [--buckets 4] [--out report.json]
                                           [--bucket-variants ID,ID,ID,ID] [--split-k]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import abi, tuned
from .tune import read_manifest

ALIGN = 4          # floats; every operand starts 16-byte aligned


def batch_shapes(count=2000, seed=0, lo=16, hi=1024, step=16):
    """[(M, N, K)]: each log-uniform on [lo, hi], rounded to the nearest
    multiple of `step` and clamped to [lo, hi]."""
    rng = np.random.default_rng([4, seed])
    x = np.exp(rng.uniform(math.log(lo), math.log(hi), (count, 3)))
    x = np.clip(np.rint(x / step) * step, lo, hi).astype(np.int64)
    return [tuple(int(v) for v in r) for r in x]


def bucket_members(shapes, bucket_of, b):
    """Problems of bucket b in the order their tiles enter the work list:
    K descending (a tile's work is proportional to K), then M*N descending.
    Work-group w takes tiles w, w + G, ... of the list, so the heavy tiles
    are dealt out first and the light ones even out the end of the launch
    (longest-processing-time-first), instead of a random order leaving
    some work-groups with several heavy tiles at the end."""
    idx = [i for i in range(len(shapes)) if bucket_of[i] == b]
    return sorted(idx, key=lambda i: (-shapes[i][2], -shapes[i][0] * shapes[i][1], i))


def buckets_of(shapes, nb, split_k=False):
    """Bucket index per problem: quantiles of log(M N K), nb buckets.  With
    split_k the largest bucket is cut again at its median K (K above it goes
    to bucket nb), so that its long-K problems may take a deeper slab than
    its short-K ones: nb + 1 buckets."""
    w = np.log(np.array([m * n * k for m, n, k in shapes], dtype=np.float64))
    edges = np.quantile(w, np.linspace(0, 1, nb + 1)[1:-1]) if nb > 1 else []
    b = np.searchsorted(edges, w, side="right").astype(int)
    if split_k:
        top = b == nb - 1
        ks = np.array([k for _, _, k in shapes])
        b[top & (ks > np.median(ks[top]))] = nb
    return b


class Batch:
    """Device operands of a batch, packed in three pooled buffers."""

    def __init__(self, shapes, host_ops=None, seed=0):
        import torch

        self.shapes = list(shapes)
        offs = {"A": [0], "B": [0], "C": [0]}
        for (M, N, K) in self.shapes:
            for key, n in (("A", M * K), ("B", K * N), ("C", M * N)):
                offs[key].append(offs[key][-1] + (n + ALIGN - 1) // ALIGN * ALIGN)
        self.off = {k: v[:-1] for k, v in offs.items()}
        if host_ops is None:
            g = torch.Generator(device="cuda")
            g.manual_seed(seed)
            self.A = torch.rand(offs["A"][-1], device="cuda", generator=g) * 2 - 1
            self.B = torch.rand(offs["B"][-1], device="cuda", generator=g) * 2 - 1
        else:
            a = np.zeros(offs["A"][-1], np.float32)
            b = np.zeros(offs["B"][-1], np.float32)
            for i, (A, B) in enumerate(host_ops):
                a[self.off["A"][i]:self.off["A"][i] + A.size] = A.ravel()
                b[self.off["B"][i]:self.off["B"][i] + B.size] = B.ravel()
            self.A = torch.from_numpy(a).cuda()
            self.B = torch.from_numpy(b).cuda()
        self.C = torch.zeros(offs["C"][-1], device="cuda")
        self.flops = sum(2.0 * M * N * K for M, N, K in self.shapes)

    def descs(self, idx):
        d = np.zeros(len(idx), dtype=abi.gemm_desc_dtype())
        a0, b0, c0 = self.A.data_ptr(), self.B.data_ptr(), self.C.data_ptr()
        for r, i in enumerate(idx):
            M, N, K = self.shapes[i]
            d[r] = (a0 + 4 * self.off["A"][i], b0 + 4 * self.off["B"][i], c0 + 4 * self.off["C"][i],
                    K, N, N, M, N, K, 0)
        return d

    def result(self, i):
        M, N, _ = self.shapes[i]
        o = self.off["C"][i]
        return self.C[o:o + M * N].view(M, N)


class GroupedPlan:
    """Device descriptors and prefix of one bucket for one variant."""

    def __init__(self, batch, idx, vid):
        import torch

        d = batch.descs(idx)
        self.total, prefix, self.vec = abi.sgemm_grouped_plan(vid, d)
        self.vid, self.count = vid, len(idx)
        self.d_descs = torch.from_numpy(d.view(np.uint8)).cuda()
        self.d_prefix = torch.from_numpy(prefix).cuda()

    def launch(self, alpha=1.0, beta=0.0, stream=None):
        abi.sgemm_grouped(self.vid, self.count, self.d_descs, self.d_prefix, self.total, alpha, beta,
                          self.vec, stream)


def launch_concurrent(plans, main, sides):
    """Launch every plan on its own stream: the first on `main`, the others
    on the streams `sides` (default priority), which first wait for the work
    already on `main`; `main` then waits for all of them.  The plans write
    disjoint outputs.  Captured under a graph, the fork and join become the
    graph's dependencies."""
    if len(sides) < len(plans) - 1:
        raise ValueError("one side stream per plan after the first")
    for s in sides[:len(plans) - 1]:
        s.wait_stream(main)
    plans[0].launch(stream=main)
    for p, s in zip(plans[1:], sides):
        p.launch(stream=s)
    for s in sides[:len(plans) - 1]:
        main.wait_stream(s)


def time_it(fn, reps=5, warmup=2):
    import torch

    for _ in range(warmup):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


SCREEN_PER_BUCKET = 6      # problems of each bucket checked against the FP64 reference


def screen_refs(batch, idx):
    """FP64 reference and elementwise bound (the FP32 GEMM bound) of a few
    problems of a bucket, on the device: the first, the last, the largest
    and evenly spaced ones between."""
    import torch

    pick = sorted({idx[0], idx[-1], max(idx, key=lambda i: np.prod(batch.shapes[i]))}
                  | set(idx[:: max(1, len(idx) // (SCREEN_PER_BUCKET - 3))]))[:SCREEN_PER_BUCKET]
    refs = []
    for i in pick:
        M, N, K = batch.shapes[i]
        ref = torch.empty(M * N, dtype=torch.float64, device="cuda")
        tol = torch.empty(M * N, dtype=torch.float64, device="cuda")
        abi.screen_reference(M, N, K, 1.0, batch.A.data_ptr() + 4 * batch.off["A"][i], K,
                             batch.B.data_ptr() + 4 * batch.off["B"][i], N, 0.0, None, N, ref, tol)
        refs.append((i, ref, tol))
    return refs


def screen_ok(batch, refs):
    """True when every screened problem's C meets its bound (Sec. V-C: a
    variant that gives wrong results is dropped)."""
    for i, ref, tol in refs:
        M, N, _ = batch.shapes[i]
        nbad, _ = abi.screen_compare(M, N, batch.C.data_ptr() + 4 * batch.off["C"][i], N, ref, tol)
        if nbad:
            return False
    return True


def tune_buckets(batch, bucket_of, nb, candidates, log=print):
    """Fastest grouped variant per bucket among those whose results pass the
    screen: {bucket: (vid, ms)}."""
    best = {}
    for b in range(nb):
        idx = bucket_members(batch.shapes, bucket_of, b)
        if not idx:
            continue
        refs = screen_refs(batch, idx)
        res = []
        dropped = 0
        for vid in candidates:
            plan = GroupedPlan(batch, idx, vid)
            batch.C.fill_(float("nan"))
            plan.launch()
            if not screen_ok(batch, refs):
                dropped += 1
                continue
            res.append((time_it(plan.launch, reps=3, warmup=1), vid))
        if not res:
            raise RuntimeError(f"bucket {b}: no candidate passed the screen")
        if dropped:
            log(f"[batched] bucket {b}: {dropped} candidates dropped by the screen")
        res.sort()
        best[b] = (res[0][1], res[0][0])
        log(f"[batched] bucket {b}: {len(idx)} problems, best variant {res[0][1]} "
            f"({res[0][0] * 1e3:.1f} us), median candidate {res[len(res) // 2][0] * 1e3:.1f} us")
    return best


def run(count=2000, nb=4, seed=0, log=print, bucket_variants=None, split_k=False):
    """Tune the bucket variants (or take ``bucket_variants``, one id per
    bucket), check the grouped launches on a few problems per bucket against
    the FP64 reference, then time per-problem launches, grouped launches and
    the graph."""
    import torch

    abi.variant_manifest_load(tuned.VARIANT_DIR)
    fp32 = [vid for vid, _, prec in read_manifest(with_prec=True) if prec == 0]
    shapes = batch_shapes(count, seed)
    batch = Batch(shapes, seed=seed)
    bucket_of = buckets_of(shapes, nb, split_k)
    nb = int(bucket_of.max()) + 1
    t0 = time.perf_counter()
    if bucket_variants is None:
        best = tune_buckets(batch, bucket_of, nb, fp32, log)
    else:
        if len(bucket_variants) != nb or any(v not in fp32 for v in bucket_variants):
            raise ValueError(f"need {nb} FP32 variant ids, one per bucket")
        best = {b: (v, float("nan")) for b, v in enumerate(bucket_variants) if np.any(bucket_of == b)}
    tune_s = time.perf_counter() - t0
    plans = [GroupedPlan(batch, bucket_members(shapes, bucket_of, b), best[b][0]) for b in sorted(best)]
    stream = torch.cuda.current_stream()

    def grouped():
        for p in plans:
            p.launch(stream=stream)

    def per_problem():
        for i, (M, N, K) in enumerate(shapes):
            o = batch.off
            abi.sgemm_variant(best[bucket_of[i]][0], M, N, K, 1.0, batch.A.data_ptr() + 4 * o["A"][i], K,
                              batch.B.data_ptr() + 4 * o["B"][i], N, 0.0, batch.C.data_ptr() + 4 * o["C"][i], N,
                              stream)

    # The grouped launches' results on the screened problems of every bucket.
    refs = [r for b in sorted(best) for r in screen_refs(batch, bucket_members(shapes, bucket_of, b))]
    batch.C.fill_(float("nan"))
    grouped()
    if not screen_ok(batch, refs):
        raise RuntimeError("grouped launches fail the screen")
    ms_single = time_it(per_problem, reps=3, warmup=1)
    ms_grouped = time_it(grouped, reps=10, warmup=2)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        grouped()                        # warm the side stream before capture
    stream.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        for p in plans:
            p.launch(stream=torch.cuda.current_stream())
    ms_graph = time_it(graph.replay, reps=20, warmup=2)

    # The same launches on concurrent streams, the largest bucket first.
    largest_first = plans[::-1]
    sides = [torch.cuda.Stream() for _ in largest_first[1:]]

    def concurrent():
        launch_concurrent(largest_first, torch.cuda.current_stream(), sides)

    batch.C.fill_(float("nan"))
    concurrent()
    if not screen_ok(batch, refs):
        raise RuntimeError("concurrent grouped launches fail the screen")
    ms_concurrent = time_it(concurrent, reps=10, warmup=2)
    graph_c = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        launch_concurrent(largest_first, side, sides)    # warm the streams before capture
    stream.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph_c):
        launch_concurrent(largest_first, torch.cuda.current_stream(), sides)
    batch.C.fill_(float("nan"))
    graph_c.replay()
    if not screen_ok(batch, refs):
        raise RuntimeError("the concurrent graph fails the screen")
    ms_graph_c = time_it(graph_c.replay, reps=20, warmup=2)
    tf = lambda ms: batch.flops / ms / 1e9  # noqa: E731
    rep = {"count": count, "buckets": nb, "split_k": split_k, "seed": seed, "gflop": batch.flops / 1e9,
           "algorithmic_gbytes": sum(4.0 * (M * K + K * N + M * N) for M, N, K in shapes) / 1e9,
           "bucket_variants": {str(b): {"variant": v, "name": abi.variant_info(v).split()[1], "ms": ms,
                                        "problems": int(np.sum(bucket_of == b))}
                               for b, (v, ms) in best.items()},
           "ms_per_problem_launches": ms_single, "ms_grouped": ms_grouped, "ms_grouped_graph": ms_graph,
           "tflops_per_problem_launches": tf(ms_single), "tflops_grouped": tf(ms_grouped),
           "tflops_grouped_graph": tf(ms_graph), "ms_concurrent": ms_concurrent,
           "ms_concurrent_graph": ms_graph_c, "tflops_concurrent": tf(ms_concurrent),
           "tflops_concurrent_graph": tf(ms_graph_c), "bucket_tuning_seconds": tune_s,
           "screened_problems": len(refs)}
    log(f"[batched] {count} GEMMs, {rep['gflop']:.1f} GFLOP: per-problem launches {ms_single:.3f} ms "
        f"({tf(ms_single):.1f} TFLOP/s), grouped {ms_grouped:.3f} ms ({tf(ms_grouped):.1f}), "
        f"grouped in a graph {ms_graph:.3f} ms ({tf(ms_graph):.1f}), concurrent streams {ms_concurrent:.3f} ms "
        f"({tf(ms_concurrent):.1f}), concurrent in a graph {ms_graph_c:.3f} ms ({tf(ms_graph_c):.1f})")
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--buckets", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--bucket-variants", default=None,
                    help="comma-separated variant ids, one per bucket (skips the bucket tuning)")
    ap.add_argument("--split-k", action="store_true",
                    help="cut the largest size bucket again at its median K (one more bucket)")
    args = ap.parse_args(argv)
    bv = [int(x) for x in args.bucket_variants.split(",")] if args.bucket_variants else None
    rep = run(args.count, args.buckets, args.seed, log=lambda s: print(s, flush=True), bucket_variants=bv,
              split_k=args.split_k)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
