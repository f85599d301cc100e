"""Pins of the portability-tuning oracle against the paper's printed numbers,
hand-derived small cases, and invariants of the definitions."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import ptune_ref as pr
from paper_2507_15277_amd import datagen

INF = float("inf")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table_vi.txt")


def _table_vi():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            d, M, N, K, t, slow, speed = line.split()
            rows.append((d, int(M), int(N), int(K), float(t), float(slow), float(speed)))
    return rows


def test_table_vi_quadro_pair():
    # Table VI (Sec. V-C): two Quadro rows share input (1024,1024,256).  The
    # faster (0.157 ms) has slowdown 1.0, so it is the best; the worst is
    # implied by its speedup 474.71.  The other row's printed slowdown and
    # speedup are then independent checks of the post-processing formulas.
    rows = [r for r in _table_vi() if r[0] == "Quadro"]
    slow_row, best_row = rows
    worst = best_row[4] * best_row[6]
    times = [[best_row[4]], [slow_row[4]], [worst]]
    best, wst, best_id, slowdown, speedup = pr.postprocess(times)
    assert best_id == [0] and best == [0.157]
    assert round(slowdown[1][0], 2) == slow_row[5]          # 4.41
    assert round(speedup[1][0], 2) == slow_row[6]           # 107.55
    assert round(slowdown[0][0], 2) == best_row[5]          # 1.0
    assert round(speedup[0][0], 2) == best_row[6]           # 474.71
    assert slowdown[2][0] == pytest.approx(worst / 0.157) and speedup[2][0] == 1.0


def test_table_vi_vega_rows_consistent():
    # Each Vega row fixes best = t/slowdown and worst = t*speedup; feeding
    # those back must reproduce the printed ratios to the printed precision.
    for d, M, N, K, t, slow, speed in [r for r in _table_vi() if r[0] == "Vega"]:
        times = [[t / slow], [t], [t * speed]]
        _, _, _, slowdown, speedup = pr.postprocess(times)
        assert round(slowdown[1][0], 2) == slow
        assert round(speedup[1][0], 2) == speed


def test_search_cost_count():
    # Sec. IV-C-1: 1,343 Quadro variants, best 3 on 10 inputs needs
    # "over 24 billion" evaluations under the |iota||delta||eps||K|^|kappa| bound.
    n = pr.search_evaluations(10, 1, 1, 1343, 3)
    assert n == 24_223_006_070
    assert 24e9 < n < 25e9


def test_hand_example():
    # 3 variants x 2 shapes, worked by hand:
    #   t = [[1, 4], [1.5, 1.5], [4, 1]], best = [1, 1]
    #   k=1: v0 -> sqrt(1*4)=2, v1 -> sqrt(1.5*1.5)=1.5, v2 -> 2  => {1}, 1.5
    #   k=2: {0,2} -> 1; {0,1} -> sqrt(1*1.5); {1,2} -> sqrt(1.5*1) => {0,2}, 1
    t = [[1.0, 4.0], [1.5, 1.5], [4.0, 1.0]]
    assert pr.portability_tune(t, 1) == ((1,), pytest.approx(1.5))
    assert pr.portability_tune(t, 2) == ((0, 2), 1.0)
    assert pr.library_cost(t, (0, 1)) == pytest.approx(math.sqrt(1.5))
    assert pr.fraction_of_best(t, (1,)) == pytest.approx(1 / 1.5)


def _block_table(groups, n_filler=3):
    """Variant g is best (t=1) exactly on group g's shapes and 2 elsewhere;
    filler variants are 3 everywhere.  Known answer by construction."""
    ns = sum(groups)
    owner = []
    for g, n in enumerate(groups):
        owner += [g] * n
    t = [[1.0 if owner[s] == g else 2.0 for s in range(ns)] for g in range(len(groups))]
    t += [[3.0] * ns for _ in range(n_filler)]
    return t


def test_block_structure_known_answer():
    groups = [5, 3, 2]
    t = _block_table(groups)
    ns = sum(groups)
    # k = #groups: the group owners, cost exactly 1.
    kappa, c = pr.portability_tune(t, 3)
    assert kappa == (0, 1, 2) and c == 1.0
    # k = 1: owner of the largest group; cost 2^(shapes outside / all).
    kappa, c = pr.portability_tune(t, 1)
    assert kappa == (0,) and c == pytest.approx(2.0 ** ((ns - 5) / ns))
    # k = 2: owners of the two largest groups.
    kappa, c = pr.portability_tune(t, 2)
    assert kappa == (0, 1) and c == pytest.approx(2.0 ** (2 / ns))


def test_failed_entries_are_routed_around():
    # v0 is best on both shapes it runs but failed the screen on shape 2.
    t = [[1.0, 1.0, INF], [1.2, 1.2, 1.2], [3.0, 3.0, 1.0]]
    kappa, c = pr.portability_tune(t, 1)
    assert kappa == (1,) and c == pytest.approx(1.2 ** (2 / 3) * 1.2 ** (1 / 3))
    kappa, c = pr.portability_tune(t, 2)
    assert kappa == (0, 2) and c == 1.0
    assert pr.library_cost(t, (0,)) == INF
    best, worst, best_id, slowdown, speedup = pr.postprocess(t)
    assert best_id == [0, 0, 2] and worst == [3.0, 3.0, 1.2]
    assert slowdown[0][2] == INF and speedup[0][2] == 0.0


def _rand_table(seed, nv, ns):
    rng = np.random.default_rng(seed)
    return (np.exp(rng.normal(0, 0.7, (nv, ns))) * rng.uniform(1, 5, ns)).tolist()


@pytest.mark.parametrize("seed", range(6))
def test_invariants(seed):
    nv, ns = 9, 6
    t = _rand_table(seed, nv, ns)
    costs = [pr.portability_tune(t, k)[1] for k in range(1, nv + 1)]
    # cost >= 1, non-increasing in k, and 1 once every per-shape winner fits.
    assert all(c >= 1.0 - 1e-15 for c in costs)
    assert all(costs[i + 1] <= costs[i] + 1e-15 for i in range(len(costs) - 1))
    _, _, best_id, _, _ = pr.postprocess(t)
    n_winners = len(set(best_id))
    assert costs[n_winners - 1] == pytest.approx(1.0)
    if n_winners > 1:
        assert costs[n_winners - 2] > 1.0
    # k = 1 is the variant with the smallest geomean slowdown.
    best, _, _, _, _ = pr.postprocess(t)
    g = [math.exp(np.mean([math.log(t[v][s] / best[s]) for s in range(ns)])) for v in range(nv)]
    assert pr.portability_tune(t, 1)[1] == pytest.approx(min(g))
    # Permuting shapes and variants permutes the answer and keeps the cost.
    rng = np.random.default_rng(100 + seed)
    pv, ps = rng.permutation(nv), rng.permutation(ns)
    t2 = [[t[pv[v]][ps[s]] for s in range(ns)] for v in range(nv)]
    for k in (1, 2, 3):
        k1, c1 = pr.portability_tune(t, k)
        k2, c2 = pr.portability_tune(t2, k)
        assert c2 == pytest.approx(c1, rel=1e-12)
        assert pr.library_cost(t, [pv[v] for v in k2]) == pytest.approx(c1, rel=1e-12)
    # Scaling all times of one shape by a constant changes nothing.
    t3 = [row[:] for row in t]
    for v in range(nv):
        t3[v][0] *= 7.0
    assert pr.portability_tune(t3, 2)[1] == pytest.approx(pr.portability_tune(t, 2)[1])


def test_cost_restricted_to_shapes():
    t = [[1.0, 4.0, 2.0], [2.0, 1.0, 2.0]]
    assert pr.library_cost(t, (0,), shapes=[0]) == 1.0
    assert pr.library_cost(t, (0,), shapes=[1]) == 4.0
    assert pr.library_cost(t, (1,), shapes=[0, 1]) == pytest.approx(math.sqrt(2.0))


def test_fleet_rate_eq2():
    # Two devices (2 and 1 units), two inputs (3 and 1 per task):
    # device 0: 1*3 + 2*1 = 5 -> 2/5; device 1: 4*3 + 1*1 = 13 -> 1/13.
    rate = pr.fleet_rate([[1.0, 2.0], [4.0, 1.0]], [2, 1], [3, 1])
    assert rate == pytest.approx(2 / 5 + 1 / 13)


def test_checkerboard_split():
    train, held = datagen.checkerboard_split()
    assert len(train) == 14 and len(held) == 13
    assert set(train) | set(held) == set(datagen.grid27())
    corners = [s for s in itertools.product((256, 4096), repeat=3)]
    assert all(c in train for c in corners)
    assert (1024, 1024, 1024) in held
    assert sum(1 for s in train if s.count(1024) == 2) == 6
    assert all(s.count(1024) == 1 for s in held if s != (1024, 1024, 1024))


def test_nearest_shape_hand_cases():
    train, held = datagen.checkerboard_split()
    # Every training shape is nearest to itself.
    for i, s in enumerate(train):
        assert pr.nearest_training_shape(train, *s) == i
    # (256,256,1024): distance 2 to (256,256,256) and to (256,256,4096);
    # the first of them is (256,256,256).
    assert train[pr.nearest_training_shape(train, 256, 256, 1024)] == (256, 256, 256)
    # 1024^3: distance 2 to each of the six two-1024 shapes; the first is
    # (256,1024,1024).
    assert train[pr.nearest_training_shape(train, 1024, 1024, 1024)] == (256, 1024, 1024)
    # (4096,4096,1024): distance 2 to (1024,4096,1024), (4096,1024,1024),
    # (4096,4096,256) and (4096,4096,4096), nothing closer; the first of
    # these in lexicographic order is (1024,4096,1024).
    assert train[pr.nearest_training_shape(train, 4096, 4096, 1024)] == (1024, 4096, 1024)
    # (512,4096,4096): distance 1 to (256,4096,4096).
    assert train[pr.nearest_training_shape(train, 512, 4096, 4096)] == (256, 4096, 4096)
    # Degenerate sizes are clamped to 1.
    assert train[pr.nearest_training_shape(train, 0, 1, 1)] == (256, 256, 256)


def test_dispatch_vote_hand_cases():
    train, _ = datagen.checkerboard_split()
    members = [7, 3, 9]
    # Member 3 is the winner (cost 0) on the six two-1024 shapes except
    # (256,1024,1024), where member 7 wins; member 9 wins the corners.
    cost = []
    for s in train:
        if s == (256, 1024, 1024):
            cost.append([0.0, 0.5, 2.0])
        elif s.count(1024) == 2:
            cost.append([0.4, 0.0, 2.0])
        else:
            cost.append([1.0, 1.0, 0.0])
    # A training shape gets its own winner.
    assert pr.dispatch(train, members, cost, 256, 1024, 1024) == 7
    assert pr.dispatch(train, members, cost, 1024, 1024, 256) == 3
    assert pr.dispatch(train, members, cost, 4096, 4096, 4096) == 9
    # 1024^3: the six two-1024 shapes vote; totals 7: 0+5*0.4 = 2.0,
    # 3: 0.5+0 = 0.5, 9: 12 -> member 3 (the nearest-first rule alone would
    # have taken 7, the winner of (256,1024,1024)).
    assert pr.dispatch(train, members, cost, 1024, 1024, 1024) == 3
    # (256,256,1024): four shapes at distance 2 vote: the corners
    # (256,256,256) and (256,256,4096) [1, 1, 0] each, (256,1024,1024)
    # [0, 0.5, 2] and (1024,256,1024) [0.4, 0, 2]; totals 2.4, 2.5, 4.0 ->
    # member 7.
    assert pr.dispatch(train, members, cost, 256, 256, 1024) == 7
    # (256,256,2048): distance 1 to (256,256,4096) only -> its winner, 9.
    assert pr.dispatch(train, members, cost, 256, 256, 2048) == 9
    # Equal totals go to the member listed first: two members identical.
    cost2 = [[0.3, 0.3, 1.0] for _ in train]
    assert pr.dispatch(train, members, cost2, 1024, 1024, 1024) == 7
    # A member that failed on one of the nearest shapes cannot win there
    # unless every member did.
    cost3 = [[INF if s == (256, 1024, 1024) else 0.0, 0.1, 0.2] for s in train]
    assert pr.dispatch(train, members, cost3, 1024, 1024, 1024) == 3
    cost4 = [[INF, INF, INF] if s == (256, 1024, 1024) else [0.5, 0.1, 0.2] for s in train]
    assert pr.dispatch(train, members, cost4, 1024, 1024, 1024) == 7


def test_wave_efficiency_closed_forms():
    # One full wave, a partial first wave, one group past a full wave, and
    # several full waves: groups / (ceil(groups / cus) * cus).
    assert pr.wave_efficiency(256, 256) == 1.0
    assert pr.wave_efficiency(64, 256) == 0.25
    assert pr.wave_efficiency(257, 256) == 257 / 512
    assert pr.wave_efficiency(1024, 256) == 1.0
    assert pr.wave_efficiency(1, 256) == 1 / 256
    assert pr.wave_efficiency(0, 256) == 1.0        # empty product: no launch
    # Never above 1, never below 1/2 once there is more than one wave.
    for g in range(257, 2000, 7):
        assert 0.5 < pr.wave_efficiency(g, 256) <= 1.0


def _groups(table, train, members, q):
    gt = [[table[(j, s)] for j in range(len(members))] for s in train]
    gq = [table[(j, q)] for j in range(len(members))]
    return gt, gq


def test_dispatch_wave_correction_hand_cases():
    train, _ = datagen.checkerboard_split()
    members = [7, 3]
    q = (1024, 1024, 1024)          # six nearest training shapes, the two-1024 ones
    near = [s for s in train if s.count(1024) == 2]
    assert len(near) == 6
    shapes = train + [q]
    # Member 3 is the per-shape best everywhere (cost 0) and member 7 is
    # 0.3 behind; member 7 launches 1024 groups on every shape (E = 1).
    cost = [[0.3, 0.0] for _ in train]
    # (a) Member 3 fills the device (512 groups, E = 1) on every training
    # shape but launches only 64 groups at q (E = 1/4): its six corrections
    # are log 1 - log(1/4) = log 4, total 6 log 4 = 8.32 > 6 * 0.3 = 1.8 -> 7.
    tab = {(0, s): 1024 for s in shapes}
    tab.update({(1, s): 512 for s in train})
    tab[(1, q)] = 64
    gt, gq = _groups(tab, train, members, q)
    assert pr.dispatch(train, members, cost, *q) == 3                     # plain vote
    assert pr.dispatch(train, members, cost, *q, gt, gq, 256) == 7
    # (b) The reverse: member 3 is 0.5 behind everywhere but launched only
    # 128 groups (E = 1/2) on the training shapes and fills the device at q:
    # each term 0.5 + log(1/2) - log 1 = -0.193, total -1.16 < 0 -> 3.
    cost_b = [[0.0, 0.5] for _ in train]
    tab_b = {(0, s): 256 for s in shapes}
    tab_b.update({(1, s): 128 for s in train})
    tab_b[(1, q)] = 256
    gt, gq = _groups(tab_b, train, members, q)
    assert pr.dispatch(train, members, cost_b, *q) == 7
    assert pr.dispatch(train, members, cost_b, *q, gt, gq, 256) == 3
    # With cus = 0 or no groups the correction is off.
    assert pr.dispatch(train, members, cost_b, *q, gt, gq, 0) == 7
    assert pr.dispatch(train, members, cost_b, *q, None, gq, 256) == 7
    # (c) A training shape keeps its own winner whatever the groups, as its
    # launch at the query is the same launch.
    s0 = (256, 1024, 1024)
    tab_c = dict(tab)
    tab_c[(0, s0)] = 3
    tab_c[(1, s0)] = 5000
    gt, gq = _groups(tab_c, train, members, s0)
    assert pr.dispatch(train, members, cost, *s0, gt, gq, 256) == 3


def test_dispatch_wave_correction_vanishes_on_full_waves():
    # When every launch is a whole number of full waves, E = 1 everywhere and
    # the corrected rule is the plain vote, for any costs and query.
    rng = np.random.default_rng(5)
    train, _ = datagen.checkerboard_split()
    members = [11, 4, 8, 2]
    for _ in range(20):
        cost = rng.exponential(0.3, (len(train), len(members))).tolist()
        gt = (rng.integers(1, 9, (len(train), len(members))) * 256).tolist()
        gq = (rng.integers(1, 9, len(members)) * 256).tolist()
        q = tuple(int(x) for x in 2 ** rng.integers(6, 14, 3))
        assert pr.dispatch(train, members, cost, *q, gt, gq, 256) == pr.dispatch(train, members, cost, *q)


def test_assign_winners():
    t = [[1.0, 5.0, 2.0], [2.0, 1.0, 2.0], [3.0, 3.0, 1.0]]
    assert pr.assign_winners(t, (0, 1), [0, 1, 2]) == [0, 1, 0]
    assert pr.assign_winners(t, (1, 2), [0, 2]) == [1, 2]


# --- Eq. 2 on one device, k-means and decision-tree selectors -------------------

def test_total_time_is_the_reciprocal_fleet_rate():
    # One device: Eq. 2's rate is quantity(d) / sum_i y' quantity(i) with
    # y' the set's best time, so the subset maximising the rate minimises
    # the weighted total time.
    t = _rand_table(11, 7, 5)
    w = [3.0, 1.0, 2.0, 5.0, 1.0]
    rates = {}
    for kap in itertools.combinations(range(7), 2):
        y = [[min(t[v][s] for v in kap) for s in range(5)]]
        rates[kap] = pr.fleet_rate(y, [4], w)
        assert rates[kap] == pytest.approx(4.0 / pr.total_time(t, kap, range(5), w))
    best_rate = max(rates, key=lambda k: (rates[k], [-x for x in k]))
    kap, tot = pr.portability_tune_total(t, 2, range(5), w)
    assert kap == best_rate


def test_total_time_hand_example():
    # Shape 0 costs 100x more than shape 1: the total-time objective keeps
    # the variant that is fastest on shape 0 even though it is 4x slower on
    # shape 1, where Eq. 1 (geomean) prefers the balanced variant.
    t = [[100.0, 4.0], [110.0, 1.0]]
    assert pr.portability_tune_total(t, 1, [0, 1], [1.0, 1.0]) == ((0,), 104.0)
    assert pr.portability_tune(t, 1)[0] == (1,)


def test_kmeans_closed_forms():
    t = _rand_table(12, 6, 5)
    pts = pr.performance_vectors(t, range(5))
    # k = 1: the single centroid is the mean vector; its best variant.
    mean = np.mean(np.array(pts), axis=0)
    kap, assign, _ = pr.kmeans_select(t, 1, list(range(5)), [0])
    assert kap == (int(np.argmax(mean)),) and assign == [0] * 5
    # k = #shapes, seeded on every shape: each shape its own cluster, so the
    # set holds every per-shape winner (made distinct).
    kap, assign, it = pr.kmeans_select(t, 5, list(range(5)), [0, 1, 2, 3, 4])
    assert assign == [0, 1, 2, 3, 4] and it == 2
    _, _, best_id, _, _ = pr.postprocess(t)
    assert set(best_id) <= set(kap)


def test_kmeans_two_groups():
    # Shapes 0-2 want variant 0, shapes 3-5 variant 1; started from one shape
    # of each group, Lloyd's algorithm separates them.
    t = [[1.0, 1.0, 1.0, 3.0, 3.0, 3.0], [3.0, 3.0, 3.0, 1.0, 1.0, 1.0], [2.0] * 6]
    kap, assign, _ = pr.kmeans_select(t, 2, list(range(6)), [0, 3])
    assert kap == (0, 1) and assign == [0, 0, 0, 1, 1, 1]


def test_tree_closed_forms():
    t = [[1.0, 1.0, 1.0, 3.0, 3.0, 3.0], [3.0, 3.0, 3.0, 1.0, 1.0, 1.0], [2.0] * 6]
    feats = [[8.0], [9.0], [10.0], [11.0], [12.0], [13.0]]
    # One split at 10.5 separates the two groups exactly.
    kap, leaf = pr.tree_select(t, 2, list(range(6)), feats)
    assert kap == (0, 1) and leaf == [0, 0, 0, 1, 1, 1]
    # k = 1: the root's mean vector (0.667, 0.667, 0.5): ties -> variant 0.
    kap, leaf = pr.tree_select(t, 1, list(range(6)), feats)
    assert kap == (0,) and leaf == [0] * 6


def test_tree_model_routes_like_its_splits():
    # One feature; variant 0 is best on features 8, 9, variant 1 on 10, 11,
    # variant 2 on 12, 13.  The root's best splits, 9.5 and 11.5, lower the
    # squared error equally (each isolates one identical pair), so the tie
    # goes to the lower threshold, 9.5.  Then only the right leaf {10..13}
    # gains from a split (at 11.5); its children are nodes 3 and 4.
    t = [[1.0, 1.0, 3.0, 3.0, 3.0, 3.0],
         [3.0, 3.0, 1.0, 1.0, 3.0, 3.0],
         [3.0, 3.0, 3.0, 3.0, 1.0, 1.0]]
    feats = [[8.0], [9.0], [10.0], [11.0], [12.0], [13.0]]
    kap, leaf, nodes, each = pr.tree_model(t, 3, list(range(6)), feats)
    assert kap == (0, 1, 2) and leaf == [0, 0, 1, 1, 2, 2] and each == [0, 1, 2]
    assert nodes == [(0, 9.5, 1, 2), (-1, 0.0, 0, -1), (0, 11.5, 3, 4), (-1, 0.0, 1, -1), (-1, 0.0, 2, -1)]
    assert pr.tree_route(nodes, [9.5]) == 0            # thresholds are inclusive on the left
    assert pr.tree_route(nodes, [9.6]) == 1
    assert pr.tree_route(nodes, [11.5]) == 1
    assert pr.tree_route(nodes, [-3.0]) == 0 and pr.tree_route(nodes, [40.0]) == 2
    # k = 1: one leaf; every point routes to it.
    kap, leaf, nodes, each = pr.tree_model(t, 1, list(range(6)), feats)
    assert nodes == [(-1, 0.0, 0, -1)] and pr.tree_route(nodes, [100.0]) == 0


def test_tree_model_routes_training_points_to_their_leaves():
    rng = np.random.default_rng(17)
    for _ in range(10):
        t = rng.uniform(1.0, 5.0, (6, 12)).tolist()
        feats = rng.integers(0, 5, (12, 3)).astype(float).tolist()
        for k in (1, 2, 3, 5):
            kap, leaf, nodes, each = pr.tree_model(t, k, list(range(12)), feats)
            assert len(nodes) == 2 * (max(leaf) + 1) - 1
            assert sorted(each) == list(kap)
            for i in range(12):
                assert pr.tree_route(nodes, feats[i]) == leaf[i]

