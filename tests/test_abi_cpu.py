"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before touching HIP, parses set files,
and its host-side portability tuning agrees with the oracle."""
import itertools
import os
import re

import numpy as np
import pytest

from oracle import ptune_ref as pr
from paper_2507_15277_amd import abi, datagen, space

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fewfit.h")
INF = float("inf")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(abi.LIB_PATH):
        pytest.fail("libfewfit.so not built (run __graft_entry__.build())")
    return abi.lib()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M))


def test_exports_every_declared_symbol(L):
    declared = _declared()
    assert declared == set(abi.EXPORTS), declared ^ set(abi.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_header_error_codes_match_binding():
    text = open(HEADER).read()
    codes = dict(re.findall(r"#define (FF_\w+) \((-?\d+)\)", text))
    for name, val in codes.items():
        assert getattr(abi, name) == int(val), name


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), abi.FF_ERR_M),
    ((4, -1, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), abi.FF_ERR_N),
    ((4, 4, -1, 1.0, 8, 4, 8, 4, 0.0, 8, 4), abi.FF_ERR_K),
    ((4, 4, 4, 1.0, None, 4, 8, 4, 0.0, 8, 4), abi.FF_ERR_A),
    ((4, 4, 4, 1.0, 8, 3, 8, 4, 0.0, 8, 4), abi.FF_ERR_LDA),
    ((4, 4, 4, 1.0, 8, 4, None, 4, 0.0, 8, 4), abi.FF_ERR_B),
    ((4, 4, 4, 1.0, 8, 4, 8, 3, 0.0, 8, 4), abi.FF_ERR_LDB),
    ((4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, None, 4), abi.FF_ERR_C),
    ((4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 3), abi.FF_ERR_LDC),
    ((4, 4, 0, 1.0, 8, 0, 8, 4, 0.0, 8, 4), abi.FF_ERR_LDA),   # lda >= max(1, K)
    ((2 ** 31, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), abi.FF_ERR_TOO_LARGE),
])
def test_argument_errors_before_any_hip_call(L, args, code):
    M, N, K, al, A, lda, B, ldb, be, C, ldc = args
    rc = L.sgemm(M, N, K, al, A, lda, B, ldb, be, C, ldc, None)
    assert rc == code, abi.last_error()
    rc = L.sgemm_variant(0, M, N, K, al, A, lda, B, ldb, be, C, ldc, None)
    assert rc == code


def test_null_operands_allowed_when_not_read(L):
    # alpha == 0 and beta == 1, or M == 0: quick return with NULL A/B.
    assert L.sgemm(4, 4, 4, 0.0, None, 4, None, 4, 1.0, 8, 4, None) == 0
    assert L.sgemm(0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, None) == 0
    assert L.sgemm(4, 4, 0, 1.0, None, 1, None, 4, 1.0, 8, 4, None) == 0


def test_form_arguments(L):
    assert L.sgemm_form(7, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4, None) == abi.FF_ERR_ARG
    assert L.sgemm_form(-1, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4, None) == abi.FF_ERR_ARG
    assert L.variant_select_form(6, 1, 1, 1) == abi.FF_ERR_ARG
    assert L.variant_select_form(abi.FF_FORM_MIXED, 1, 1, 1) == abi.FF_ERR_NO_SET
    assert L.variant_select_form(2, 1, 1, 1) == abi.FF_ERR_NO_SET
    assert L.variant_select_form(4, 1, 1, 1) == abi.FF_ERR_NO_SET
    assert L.sgemm_form(1, -1, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4, None) == abi.FF_ERR_M


def test_no_set_loaded(L):
    assert L.variant_select(256, 256, 256) == abi.FF_ERR_NO_SET
    assert L.sgemm(4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4, None) == abi.FF_ERR_NO_SET
    assert L.variant_select(-1, 1, 1) == abi.FF_ERR_M
    assert L.sgemm_variant(10 ** 6, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4, None) == abi.FF_ERR_VARIANT


GOOD_VARIANT = space.DEFAULT.descriptor(0)


@pytest.mark.parametrize("body,code", [
    ("", abi.FF_ERR_PARSE),
    ("fewfit-set 2\n", abi.FF_ERR_PARSE),
    ("fewfit-set 1\narch gfx950\ncodedir .\nvariant 0 bad\nrule 1 1 1 0 0\nend\n", abi.FF_ERR_PARSE),
    (f"fewfit-set 1\narch gfx950\ncodedir .\nvariant {GOOD_VARIANT}\nrule 1 1 1 5 0\nend\n", abi.FF_ERR_PARSE),
    (f"fewfit-set 1\narch gfx950\ncodedir .\nvariant {GOOD_VARIANT}\nrule 1 1 1 0 0\n", abi.FF_ERR_PARSE),
    (f"fewfit-set 1\narch gfx950\ncodedir .\nvariant {GOOD_VARIANT}\nend\n", abi.FF_ERR_PARSE),
    (f"fewfit-set 1\narch gfx950\ncodedir .\nvariant {GOOD_VARIANT}\nvariant {GOOD_VARIANT}\n"
     "rule 1 1 1 0 0 0\nend\n", abi.FF_ERR_PARSE),
    (f"fewfit-set 1\narch gfx950\ncodedir .\nvariant {GOOD_VARIANT}\nrule 1 1 1 0 0 9\nend\n", abi.FF_ERR_PARSE),
    (f"fewfit-set 1\narch gfx950\ncodedir .\nvariant {GOOD_VARIANT}\nrule 1 1 1 0\nend\n", abi.FF_ERR_PARSE),
    (f"fewfit-set 1\narch gfx950\ncodedir .\nvariant {GOOD_VARIANT}\nrule 1 1 1 0 -1\nend\n", abi.FF_ERR_PARSE),
    (f"fewfit-set 1\narch gfx950\ncodedir .\nvariant {GOOD_VARIANT}\nrule 1 1 1 0 x\nend\n", abi.FF_ERR_PARSE),
    (f"fewfit-set 1\nfoo 1\nend\n", abi.FF_ERR_PARSE),
    # a split-precision descriptor must not carry split-K groups
    ("fewfit-set 1\narch gfx950\ncodedir .\nform bf16x3\nvariant 5 x 64 64 32 32 2 2 2 4 1 8 1 1\n"
     "rule 1 1 1 5 0\nend\n", abi.FF_ERR_PARSE),
    # members must match the set's form
    (f"fewfit-set 1\narch gfx950\ncodedir .\nform bf16x6\nvariant {GOOD_VARIANT}\nrule 1 1 1 0 0\nend\n",
     abi.FF_ERR_PARSE),
    (f"fewfit-set 1\narch gfx950\ncodedir .\nform fp64\nvariant {GOOD_VARIANT}\nrule 1 1 1 0 0\nend\n",
     abi.FF_ERR_PARSE),
    # a form may be given once per set file
    (f"fewfit-set 1\narch gfx950\ncodedir .\nform mixed\nform mixed x\nvariant {GOOD_VARIANT}\nrule 1 1 1 0 0\n"
     "end\n", abi.FF_ERR_PARSE),
])

def test_set_file_parse_errors(L, tmp_path, body, code):
    p = tmp_path / "set.txt"
    p.write_text(body)
    assert L.variant_set_load(os.fsencode(str(p))) == code, abi.last_error()


def test_mixed_set_parses(L, tmp_path):
    # The mixed slot takes members of any form: the file parses, and only the
    # device check (no GPU here) can refuse it.
    split = "7 y 64 64 32 32 2 2 1 4 1 8 1 4 1"      # an fp16x3 descriptor
    p = tmp_path / "set.txt"
    p.write_text(f"fewfit-set 1\narch gfx950\ncodedir .\nform mixed\nvariant {GOOD_VARIANT}\nvariant {split}\n"
                 "rule 1 1 1 0 0 0.5\nend\n")
    rc = L.variant_set_load(os.fsencode(str(p)))
    assert rc != abi.FF_ERR_PARSE, abi.last_error()
    # The same members under a single form are refused.
    p.write_text(p.read_text().replace("form mixed", "form fp32"))
    assert L.variant_set_load(os.fsencode(str(p))) == abi.FF_ERR_PARSE


def test_set_file_missing(L, tmp_path):
    assert L.variant_set_load(os.fsencode(str(tmp_path / "nope.txt"))) == abi.FF_ERR_IO
    assert L.variant_manifest_load(os.fsencode(str(tmp_path))) == abi.FF_ERR_IO


# --- host portability tuning vs the oracle ------------------------------------

def _rand_table(seed, nv, ns, fail_frac=0.0):
    rng = np.random.default_rng([3, seed])
    t = np.exp(rng.normal(0, 0.6, (nv, ns))) * rng.uniform(0.5, 20, ns)
    if fail_frac:
        t[rng.random((nv, ns)) < fail_frac] = INF
    return t


@pytest.mark.parametrize("seed", range(8))
def test_postprocess_matches_oracle(seed):
    t = _rand_table(seed, 7, 5, fail_frac=0.15)
    best, worst, best_id, slow, speed = abi.ptune_postprocess(t)
    b2, w2, bi2, s2, sp2 = pr.postprocess(t.tolist())
    assert list(best_id) == bi2
    assert np.array_equal(best, np.array(b2)) and np.array_equal(worst, np.array(w2))
    assert np.array_equal(slow, np.array(s2)) and np.array_equal(speed, np.array(sp2))


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_exhaustive_select_matches_bruteforce(seed, k):
    nv, ns = 11, 7
    t = _rand_table(100 + seed, nv, ns, fail_frac=0.1 if seed % 2 else 0.0)
    shapes = list(range(0, ns, 1)) if seed % 3 else [0, 2, 3, 5]
    kap, cost, evals = abi.ptune_select(t, k, shapes=shapes, method=0)
    kap_ref, cost_ref = pr.portability_tune(t.tolist(), k, shapes)
    # Several sets may tie; parity is on the objective value.
    if cost_ref == INF:
        assert cost == INF
    else:
        assert cost == pytest.approx(cost_ref, rel=1e-12)
        assert pr.library_cost(t.tolist(), kap, shapes) == pytest.approx(cost, rel=1e-12)
    assert len(kap) == k and len(set(kap)) == k
    assert abi.ptune_cost(t, kap, shapes) == pytest.approx(cost, rel=1e-12) or cost == INF


@pytest.mark.parametrize("seed", range(6))
def test_greedy_swap_is_a_local_optimum(seed):
    nv, ns = 12, 8
    t = _rand_table(200 + seed, nv, ns)
    for k in (2, 3, 5):
        kap, cost, _ = abi.ptune_select(t, k, method=1)
        _, best_cost = pr.portability_tune(t.tolist(), k)
        assert cost >= best_cost * (1 - 1e-12)
        # No single swap improves the set.
        for p, v in itertools.product(range(k), range(nv)):
            if v in kap:
                continue
            trial = list(kap)
            trial[p] = v
            assert pr.library_cost(t.tolist(), trial) >= cost * (1 - 1e-12)


def test_select_known_block_answer():
    # Variant g is best (1.0) on its own group of shapes and 2.0 elsewhere;
    # three fillers at 3.0.  k = 3 must return the three owners at cost 1.
    groups = [4, 3, 2]
    owner = sum(([g] * n for g, n in enumerate(groups)), [])
    t = np.array([[1.0 if o == g else 2.0 for o in owner] for g in range(3)] + [[3.0] * 9] * 3)
    assert abi.ptune_select(t, 3, method=0)[:2] == ((0, 1, 2), 1.0)
    assert abi.ptune_select(t, 1, method=0)[0] == (0,)


def test_assign_matches_oracle():
    t = _rand_table(9, 9, 6, fail_frac=0.2)
    kap = (1, 4, 7)
    assert abi.ptune_assign(t, kap, [0, 2, 5]) == pr.assign_winners(t.tolist(), kap, [0, 2, 5])


@pytest.mark.parametrize("seed", range(5))
def test_dispatch_matches_oracle(seed):
    from paper_2507_15277_amd import datagen
    shapes = datagen.grid27()
    if seed == 0:
        train, _ = datagen.checkerboard_split()
    else:
        train, _ = datagen.random_split(seed, 14)
    rng = np.random.default_rng([4, seed])
    k = 4
    members = sorted(rng.choice(50, k, replace=False).tolist())
    cost = rng.exponential(0.3, (len(train), k))
    cost[rng.random(cost.shape) < 0.1] = INF
    for i in range(len(train)):
        cost[i, rng.integers(k)] = 0.0      # each training shape has a winner
    queries = shapes + [(512, 4096, 4096), (4096, 4096, 512), (1, 1, 1), (100, 3000, 77), (0, 5, 5)]
    for q in queries:
        assert abi.ptune_dispatch(train, members, cost, *q) == pr.dispatch(train, members, cost.tolist(), *q), q
    for i, s in enumerate(train):
        assert abi.ptune_nearest(train, *s) == i
    # With the wave correction: work-group counts from 1 to a few waves of
    # 256 compute units (and 0, an empty launch), per member and shape.
    gt = rng.integers(0, 1100, (len(train), k))
    for q in queries:
        gq = rng.integers(0, 1100, k)
        for cus in (256, 304, 0):
            got = abi.ptune_dispatch(train, members, cost, *q, gt, gq, cus)
            want = pr.dispatch(train, members, cost.tolist(), *q, gt.tolist(), gq.tolist(), cus)
            assert got == want, (q, cus)


def test_select_argument_errors():
    t = _rand_table(1, 3, 3)
    with pytest.raises(abi.FewfitError):
        abi.ptune_select(t, 0)
    with pytest.raises(abi.FewfitError):
        abi.ptune_select(t, 2, shapes=[0, 9])
    with pytest.raises(abi.FewfitError):
        abi.ptune_cost(t, [5])


@pytest.mark.parametrize("seed", range(6))
def test_total_time_select_matches_bruteforce(seed):
    nv, ns = 10, 6
    t = _rand_table(300 + seed, nv, ns, fail_frac=0.1 if seed % 2 else 0.0)
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 4.0, ns)
    shapes = list(range(ns))
    for k in (1, 2, 3):
        kap, tot, _ = abi.ptune_select_total(t, k, shapes, w, method=0)
        ref_kap, ref_tot = pr.portability_tune_total(t.tolist(), k, shapes, w.tolist())
        if ref_tot == INF:
            assert tot == INF
        else:
            assert tot == pytest.approx(ref_tot, rel=1e-12)
            assert pr.total_time(t.tolist(), kap, shapes, w.tolist()) == pytest.approx(ref_tot, rel=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_kmeans_matches_oracle(seed):
    nv, ns = 12, 9
    t = _rand_table(400 + seed, nv, ns, fail_frac=0.1 if seed % 2 else 0.0)
    rng = np.random.default_rng([5, seed])
    shapes = sorted(rng.choice(ns, 7, replace=False).tolist())
    for k in (1, 2, 3, 4):
        init = sorted(rng.choice(len(shapes), k, replace=False).tolist())
        kap, assign, it = abi.ptune_kmeans(t, k, shapes, init)
        rk, ra, rit = pr.kmeans_select(t.tolist(), k, shapes, init)
        assert kap == rk and assign == ra and it == rit


@pytest.mark.parametrize("seed", range(8))
def test_tree_matches_oracle(seed):
    from paper_2507_15277_amd import datagen
    shapes27 = datagen.grid27()
    nv = 10
    t = _rand_table(500 + seed, nv, 27)
    rng = np.random.default_rng([6, seed])
    shapes = sorted(rng.choice(27, 12, replace=False).tolist())
    feats = [[np.log2(x) for x in shapes27[s]] for s in shapes]
    for k in (1, 2, 3, 5):
        kap, leaf = abi.ptune_tree(t, k, shapes, feats)
        rk, rl = pr.tree_select(t.tolist(), k, shapes, feats)
        assert kap == rk and leaf == rl
        # The tree itself and its routing of unseen points.
        kap, leaf, nf, nt, nc, lv = abi.ptune_tree(t, k, shapes, feats, model=True)
        mk, ml, nodes, each = pr.tree_model(t.tolist(), k, shapes, feats)
        assert (kap, leaf, lv) == (mk, ml, each)
        assert [(int(nf[n]), float(nt[n]), int(nc[2 * n]), int(nc[2 * n + 1])) for n in range(len(nodes))] == nodes
        for q in datagen.grid27() + [(512, 4096, 4096), (100, 3000, 77)]:
            x = [float(np.log2(v)) for v in q]
            assert abi.ptune_tree_route(nf, nt, nc, x) == pr.tree_route(nodes, x), q


def test_manifest_matches_family():
    # The manifest lists the compiled family in order: FP32 variants first,
    # then the split-precision forms, each with its precision field.
    from paper_2507_15277_amd.tune import read_manifest
    fam = space.full_family()
    man = read_manifest(with_prec=True)
    assert [(i, v.name, v.prec) for i, v in enumerate(fam)] == man
    assert man[0][1] == space.DEFAULT.name


def test_committed_sets_match_manifest():
    """Every member line of a committed set file repeats the manifest's
    descriptor of that id, so a rebuilt family cannot leave a stale set."""
    from paper_2507_15277_amd import tuned

    man = {}
    for line in open(os.path.join(tuned.VARIANT_DIR, "manifest.txt")):
        if line.strip() and not line.startswith("#"):
            man[int(line.split()[0])] = line.split()
    sets_dir = os.path.dirname(tuned.set_path(4))
    files = sorted(f for f in os.listdir(sets_dir) if f.endswith(".txt"))
    assert files
    for fn in files:
        members = [ln.split()[1:] for ln in open(os.path.join(sets_dir, fn)) if ln.startswith("variant ")]
        assert members, fn
        for m in members:
            assert man[int(m[0])] == m, (fn, m)


def test_evaluate_slowdown_histogram():
    # portability.evaluate on a random table over the real family: the S/O
    # histogram counts every shape once, its maximum is the largest ratio of
    # the dispatched member's time to the per-shape best, and a set holding
    # every shape's winner, dispatched on its own training shapes, is at 1.
    from paper_2507_15277_amd import portability
    nv = len(portability.read_variants())
    shapes = datagen.grid27()
    rng = np.random.default_rng(77)
    t = np.exp(rng.normal(0, 0.5, (nv, len(shapes))))
    train, _ = datagen.checkerboard_split(shapes)
    train_idx = [shapes.index(s) for s in train]
    kap, _, _ = abi.ptune_select(t, 4, shapes=train_idx, method=-1)
    ev = portability.evaluate(t, shapes, train_idx, kap)
    assert sum(ev["so_hist"]["counts"]) == len(shapes)
    so = [r["frac"] for r in ev["per_shape"]]
    assert ev["so_max"] == pytest.approx(1.0 / min(so))
    winners = sorted({int(np.argmin(t[:, j])) for j in range(len(shapes))})
    ev_all = portability.evaluate(t, shapes, list(range(len(shapes))), tuple(winners))
    assert ev_all["so_max"] == pytest.approx(1.0) and ev_all["so_hist"]["counts"][0] == len(shapes)


def test_fresh_shapes_recipe():
    # The shapes that chose nothing: the 37 shapes of the paper's
    # {256, 512, 1024, 4096}^3 grid off the tuning grid (each holds a 512),
    # then 20 seeded log-uniform integer shapes in [128, 8192]; none is a
    # training or held-out shape of the tuning grid.
    f = datagen.fresh_shapes()
    assert len(f) == 57 and len(set(f)) == 57
    assert all(512 in s for s in f[:37])
    assert not set(f) & set(datagen.grid27())
    assert all(128 <= x <= 8192 for s in f[37:] for x in s)
    assert f == datagen.fresh_shapes()


def test_fresh_report_on_a_synthetic_table():
    # portability.fresh_report with the committed sets on random times over
    # the real family: fractions are at most 1, a perfect in-set pick is at
    # least the dispatched pick, and the S/O histogram counts every shape.
    from paper_2507_15277_amd import portability
    variants = portability.read_variants()
    rng = np.random.default_rng(78)
    rows = [{"M": s[0], "N": s[1], "K": s[2], "beta": 0.0, "status": "ok", "variant": v,
             "ms": float(np.exp(rng.normal(0, 0.5)))}
            for s in datagen.fresh_shapes() for v in variants if variants[v].prec == 0]
    rep = portability.fresh_report(rows, variants, log=lambda *_: None)
    assert set(rep["sets"]) == {"fixed", "k1", "k2", "k4", "k8"}
    for rec in rep["sets"].values():
        assert 0 < rec["frac_realised"] <= rec["frac_inset"] <= 1.0
        assert sum(rec["so_hist"]["counts"]) == 57
        assert rec["so_max"] == pytest.approx(1.0 / min(r["frac"] for r in rec["per_shape"]))


def test_bucket_members_order():
    # The grouped launch deals tiles out heaviest first: K descending, then
    # M*N descending, ties by problem index; every problem of the bucket
    # appears once.
    from paper_2507_15277_amd import batched
    shapes = batched.batch_shapes(300, 3)
    bucket_of = batched.buckets_of(shapes, 4)
    for b in range(4):
        idx = batched.bucket_members(shapes, bucket_of, b)
        assert sorted(idx) == [i for i in range(300) if bucket_of[i] == b]
        keys = [(-shapes[i][2], -shapes[i][0] * shapes[i][1], i) for i in idx]
        assert keys == sorted(keys)


def test_ragged_grid_recipe():
    # The unaligned counterpart of the tuning grid: every shape is a grid
    # shape moved by (1, 3, 5), so N and K are odd and no vector-load kernel
    # can run.
    r = datagen.ragged_grid()
    assert len(r) == 27 and [(m - 1, n - 3, k - 5) for m, n, k in r] == datagen.grid27()
    assert all(n % 4 and k % 4 for _, n, k in r)


def test_ragged_report_on_a_synthetic_table():
    from paper_2507_15277_amd import portability
    variants = portability.read_variants()
    rng = np.random.default_rng(79)
    shapes = datagen.grid27() + datagen.ragged_grid() + datagen.fresh_shapes()
    rows = [{"M": s[0], "N": s[1], "K": s[2], "beta": 0.0, "status": "ok", "variant": v,
             "ms": float(np.exp(rng.normal(0, 0.5)))}
            for s in shapes for v in variants if variants[v].prec == 0]
    rep = portability.ragged_report(rows, variants, log=lambda *_: None)
    for k, rec in rep["sets"].items():
        for sel in rec.values():
            assert len(sel["kappa"]) == int(k)
            assert all(0 < sel[x] <= 1.0 for x in ("heldout_aligned", "heldout_ragged", "fresh_paper_grid",
                                                 "fresh_ragged"))


def test_accuracy_report_on_a_synthetic_table():
    # FP32 variants miss the 1e-6 target on every K = 4096 shape, the fp16x3
    # variants meet it everywhere: the constrained selection must realise a
    # member that meets the target on all 27 shapes, and FP32 alone covers
    # only the shapes it meets it on.
    from paper_2507_15277_amd import portability
    variants = portability.read_variants()
    rng = np.random.default_rng(83)
    rows = []
    for s in datagen.grid27():
        for v in variants:
            p = variants[v].prec
            if p not in (0, 4):
                continue
            err = (2e-6 if s[2] == 4096 else 5e-7) if p == 0 else 3e-7
            rows.append({"M": s[0], "N": s[1], "K": s[2], "beta": 0.0, "status": "ok", "variant": v,
                         "data": "lognormal", "ms": float(np.exp(rng.normal(0.3 * (p > 0), 0.5))),
                         "err_norm": err})
    rep = portability.accuracy_report(rows, variants, log=lambda *_: None)
    assert rep["shapes_with_a_variant_meeting_target"]["fp32"] == 18
    assert rep["shapes_with_a_variant_meeting_target"]["fp16x3"] == 27
    assert rep["per_shape_best_geomean_tflops"]["fp32"] is None
    for k, sel in rep["sets"].items():
        assert len(sel["kappa"]) == int(k)
        assert sel["realised_meeting_target"] == 27 and sel["realised_max_err_norm"] <= 1e-6
        assert all(r["form"] == "fp16x3" for r in sel["per_shape"] if r["K"] == 4096)
    assert set(rep["sets"]["4"]["forms"]) == {"fp32", "fp16x3"}
    assert rep["fp32_k4_unconstrained"]["realised_meeting_target"] == 18


def test_accuracy_sweep_is_monotone_on_a_synthetic_table():
    # A looser target admits more variants, so the per-shape best can only
    # rise; every target's k = 4 set meets it on every shape it dispatches.
    from paper_2507_15277_amd import portability
    variants = portability.read_variants()
    rng = np.random.default_rng(89)
    errs = {0: 5e-7, 1: 3e-6, 2: 2e-7, 3: 2e-4, 4: 3e-7}
    rows = [{"M": s[0], "N": s[1], "K": s[2], "beta": 0.0, "status": "ok", "variant": v, "data": "lognormal",
             "ms": float(np.exp(rng.normal(-0.3 * variants[v].prec, 0.5))),
             "err_norm": errs[variants[v].prec] * (2.0 if s[2] == 4096 else 1.0)}
            for s in datagen.grid27() for v in variants]
    sweep = portability.accuracy_sweep(rows, variants, targets=(1e-3, 1e-5, 1e-6, 5e-7), log=lambda *_: None)
    best = [r["per_shape_best_geomean_tflops"] for r in sweep]
    assert all(a >= b for a, b in zip(best, best[1:])), best
    for r in sweep:
        assert r["k4_realised_meeting_target"] == 27 and r["k4_realised_max_err_norm"] <= r["target_err_norm"]


def test_accuracy_fresh_report_on_a_synthetic_table():
    # The committed mixed and FP32 sets dispatched on the fresh shapes: a
    # shape's member must be one of the set's, and the counts of shapes
    # meeting the target follow the planted errors (FP32 misses it where
    # K > 4096).
    from paper_2507_15277_amd import portability
    variants = portability.read_variants()
    rng = np.random.default_rng(97)
    rows = [{"M": s[0], "N": s[1], "K": s[2], "beta": 0.0, "status": "ok", "variant": v, "data": "lognormal",
             "ms": float(np.exp(rng.normal(0, 0.5))),
             "err_norm": (2e-6 if s[2] > 4096 else 5e-7) if variants[v].prec == 0 else 3e-7}
            for s in datagen.fresh_shapes() for v in variants]
    rep = portability.accuracy_fresh_report(rows, variants, log=lambda *_: None)
    long_k = sum(1 for s in datagen.fresh_shapes() if s[2] > 4096)
    assert long_k > 0
    fp32 = rep["sets"]["fp32_k4"]
    assert fp32["timed"] == 57 and fp32["meeting_target"] == 57 - long_k
    assert all(m["K"] > 4096 and m["form"] == "fp32" for m in fp32["missed"])
    mixed = rep["sets"]["mixed_k4"]
    assert mixed["timed"] == 57 and 0 < mixed["frac_of_best_meeting_target"] <= 1.0


def test_accuracy_training_report_on_a_synthetic_table():
    # Selections on 14 and on 64 training shapes, scored on the 20 random
    # fresh shapes: sizes and fractions in range, every member of a set.
    from paper_2507_15277_amd import portability
    variants = portability.read_variants()
    rng = np.random.default_rng(101)
    shapes = datagen.grid27() + datagen.fresh_shapes()
    rows = [{"M": s[0], "N": s[1], "K": s[2], "beta": 0.0, "status": "ok", "variant": v, "data": "lognormal",
             "ms": float(np.exp(rng.normal(0, 0.5))), "err_norm": 5e-7}
            for s in shapes for v in variants if variants[v].prec in (0, 4)]
    rep = portability.accuracy_training_report(rows, variants, log=lambda *_: None)
    assert len(rep["held_out"]) == 20
    for label, rec in rep["sets"].items():
        assert len(rec["kappa"]) == int(label[-1]) and 0 < rec["heldout_frac"] <= 1.0
        assert rec["heldout_meeting_target"] == 20 and rec["train_frac"] <= 1.0 + 1e-12
