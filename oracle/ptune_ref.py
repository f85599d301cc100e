"""Reference oracle for portability tuning -- TEST INFRASTRUCTURE ONLY.

Plain-Python statements of the host-side steps of the method, used only by
the test suite to check the native implementation.  Nothing here is fast;
everything is written to be read against the paper.

An execution-time table is a 2-D array ``t[v][s]``: variant ``v`` on shape
(input) ``s``, in any time unit; ``inf`` marks a variant that failed the
correctness screen or could not run on that shape (Sec. V-C: such data are
screened out).

Readings of the paper taken here (also listed in the design notes):

* Equation 1 prints ``max`` over the kernel set in the numerator; the text
  around Fig. 1 says a set performs like its best member on each
  environment, so the numerator is the *minimum* runtime over the selected
  set.  The cost is the geometric mean of slowdowns (>= 1), minimised.
* Ties (equal cost) are broken towards the lexicographically smallest tuple
  of variant ids, as produced by ``itertools.combinations``.
* The runtime dispatch rule for unseen shapes is not given by the paper
  (Sec. V-I lists it as a limitation); the rule taken here uses the training shapes
  nearest in (log2 M, log2 N, log2 K) under the L1 distance and, among the
  members of kappa, the one with the smallest summed log-slowdown over them
  (ties to the member listed first); a training shape gets its own winner.
  Optionally each member's log-slowdown at a training shape is moved to the
  query shape by its work-group wave efficiency (``wave_efficiency``): the
  fraction of the device's compute units that its last wave of work-groups
  keeps busy, averaged over the waves.  A member that launches too few
  work-groups to fill the device at a training shape is not blamed for it
  at a query shape where it does fill the device, and the reverse.
"""
from __future__ import annotations

import itertools
import math

INF = float("inf")


def _finite(x):
    return x == x and x != INF


# --- Sec. V-C: post-processing pass -------------------------------------------

def postprocess(times):
    """Per-shape best and worst, and each entry's slowdown and speedup.

    Sec. V-C: a post-processing pass relates every kernel's time to the best
    and the worst kernel for the same device and input.  Table VI prints the
    results as "Slowdown vs Oracle" (time / best) and "Speedup vs Worst"
    (worst / time).  Failed entries (inf) get slowdown inf and speedup 0.

    Returns ``(best, worst, best_id, slowdown, speedup)``; ``best_id`` is the
    lowest variant index attaining the best time, or -1 if none is finite.
    """
    nv = len(times)
    ns = len(times[0]) if nv else 0
    best, worst, best_id = [], [], []
    for s in range(ns):
        b, w, bi = INF, -INF, -1
        for v in range(nv):
            x = times[v][s]
            if not _finite(x):
                continue
            if x < b:
                b, bi = x, v
            if x > w:
                w = x
        best.append(b)
        worst.append(w if bi >= 0 else INF)
        best_id.append(bi)
    slowdown = [[INF] * ns for _ in range(nv)]
    speedup = [[0.0] * ns for _ in range(nv)]
    for v in range(nv):
        for s in range(ns):
            x = times[v][s]
            if _finite(x) and best_id[s] >= 0:
                slowdown[v][s] = x / best[s]
                speedup[v][s] = worst[s] / x
    return best, worst, best_id, slowdown, speedup


def autotune(times, s):
    """Sec. IV-A, AutoTune: the single best variant for one environment."""
    best, _, best_id, _, _ = postprocess([[row[s]] for row in times])
    return best_id[0]


# --- Sec. IV-D-1, Eq. 1: library cost function ---------------------------------

def library_cost(times, kappa, shapes=None):
    """Eq. 1 (min reading): geomean over shapes of best-in-kappa / best-overall.

    ``kappa`` is a collection of variant indices; ``shapes`` restricts the
    environments summarised (default: all).  Returns inf if some shape has no
    finite member of kappa.
    """
    ns = len(times[0])
    shapes = list(range(ns)) if shapes is None else list(shapes)
    best, _, _, _, _ = postprocess(times)
    logsum = 0.0
    for s in shapes:
        m = min((times[v][s] for v in kappa), default=INF)
        if not _finite(m) or not _finite(best[s]):
            return INF
        logsum += math.log(m / best[s])
    return math.exp(logsum / len(shapes))


def fraction_of_best(times, kappa, shapes=None):
    """1 / cost: the geomean fraction of the per-shape best that kappa reaches."""
    c = library_cost(times, kappa, shapes)
    return 0.0 if c == INF else 1.0 / c


# --- Sec. IV-B / IV-C-1: PortabilityTune by exhaustive search ------------------

def portability_tune(times, k, shapes=None):
    """kappa = argmin over all k-subsets of the variants of Eq. 1's cost.

    Exhaustive enumeration of the subsets of size ``min(k, #variants)``; ties
    go to the first subset in lexicographic order.  Returns
    ``(kappa_tuple, cost)``; ``cost`` is inf if no subset covers every shape.
    """
    nv = len(times)
    k = min(k, nv)
    best_set, best_cost = None, INF
    for kappa in itertools.combinations(range(nv), k):
        c = library_cost(times, kappa, shapes)
        if c < best_cost:
            best_set, best_cost = kappa, c
    if best_set is None:
        best_set = tuple(range(k))
    return best_set, best_cost


def search_evaluations(n_inputs, n_devices, n_envs, n_variants, set_size):
    """Sec. IV-C-1: evaluations bound |iota|*|delta|*|epsilon|*|K|^|kappa|."""
    return n_inputs * n_devices * n_envs * n_variants ** set_size


# --- Sec. IV-D-2, Eq. 2: fleet task rate ---------------------------------------

def fleet_rate(runtime, qty_device, qty_input):
    """Eq. 2: sum over devices of quantity(d) / sum over inputs of y' * quantity(i).

    ``runtime[d][i]`` is y', the runtime of input i on device d.
    """
    rate = 0.0
    for d, qd in enumerate(qty_device):
        total = 0.0
        for i, qi in enumerate(qty_input):
            total += runtime[d][i] * qi
        rate += qd / total
    return rate


# --- Runtime dispatch (Fig. 1 online step; the rule chosen here) --------------

def assign_winners(times, kappa, train_shapes_idx):
    """For each training shape, the member of kappa with the lowest time
    (ties to the lower variant id); -1 if no member is finite there."""
    out = []
    for s in train_shapes_idx:
        bv, bt = -1, INF
        for v in sorted(kappa):
            x = times[v][s]
            if _finite(x) and x < bt:
                bv, bt = v, x
        out.append(bv)
    return out


def nearest_training_shape(train_shapes, M, N, K):
    """Index of the training shape nearest to (M,N,K) in L1 distance over
    (log2 M, log2 N, log2 K); ties go to the lower index.  Sizes below 1 are
    treated as 1."""
    q = [math.log2(max(1, x)) for x in (M, N, K)]
    best_i, best_d = -1, INF
    for i, shp in enumerate(train_shapes):
        d = sum(abs(q[j] - math.log2(max(1, shp[j]))) for j in range(3))
        if d < best_d:
            best_i, best_d = i, d
    return best_i


def _dist(a, b):
    return sum(abs(math.log2(max(1, a[j])) - math.log2(max(1, b[j]))) for j in range(3))


def wave_efficiency(groups, cus):
    """Busy fraction of ``cus`` compute units over the waves needed to run
    ``groups`` work-groups one per unit: groups / (ceil(groups / cus) * cus).
    No work-groups (an empty problem) counts as fully efficient."""
    if groups <= 0:
        return 1.0
    waves = -(-groups // cus)
    return groups / (waves * cus)


def dispatch(train_shapes, members, cost, M, N, K, groups_train=None, groups_query=None, cus=0):
    """Variant chosen for (M,N,K).

    ``cost[i][j]`` is log(t / best) of member j on training shape i.  All
    training shapes at the smallest distance vote: the member with the
    smallest total cost over them wins (first member on ties).  If every
    member is infinite somewhere among them, the member cheapest on the
    first nearest shape is taken.

    With ``groups_train[i][j]`` (work-groups member j launches on training
    shape i), ``groups_query[j]`` (the same at (M,N,K)) and ``cus`` >= 1, the
    vote adds to each cost the wave correction
    log(wave_efficiency(groups_train[i][j])) - log(wave_efficiency(groups_query[j])),
    which is exactly 0 where the two launches have the same efficiency.
    """
    d = [_dist((M, N, K), s) for s in train_shapes]
    dmin = min(d)
    near = [i for i in range(len(train_shapes)) if d[i] <= dmin + 1e-9]
    corr = lambda i, j: 0.0  # noqa: E731
    if groups_train is not None and groups_query is not None and cus >= 1:
        corr = lambda i, j: (math.log(wave_efficiency(groups_train[i][j], cus))  # noqa: E731
                             - math.log(wave_efficiency(groups_query[j], cus)))
    totals = [sum(cost[i][j] + corr(i, j) for i in near) for j in range(len(members))]
    best_j = min(range(len(members)), key=lambda j: (totals[j], j))
    if totals[best_j] == INF:
        i0 = near[0]
        best_j = min(range(len(members)), key=lambda j: (cost[i0][j], j))
    return members[best_j]


# --- Sec. IV-D-2 with one device: weighted total time --------------------------

def total_time(times, kappa, shapes, weights):
    """sum_i weight(i) * min_{v in kappa} t[v][i]: the time of one fleet task
    on one device, the reciprocal of Eq. 2's rate up to quantity(d)."""
    tot = 0.0
    for s, w in zip(shapes, weights):
        m = min(times[v][s] for v in kappa)
        if not _finite(m):
            return INF
        tot += w * m
    return tot


def portability_tune_total(times, k, shapes, weights):
    """argmin over k-subsets of total_time (first subset in lexicographic
    order on ties)."""
    nv = len(times)
    k = min(k, nv)
    best_set, best_cost = None, INF
    for kappa in itertools.combinations(range(nv), k):
        c = total_time(times, kappa, shapes, weights)
        if c < best_cost:
            best_set, best_cost = kappa, c
    return (best_set if best_set is not None else tuple(range(k))), best_cost


# --- Sec. IV-C-2: k-means on performance vectors -------------------------------

def performance_vectors(times, shapes):
    """One point per environment (shape): its |K|-dim vector of relative
    performance best/t (0 where a variant failed).  The paper leaves the
    normalisation open; relative performance puts every shape on the same
    scale, as Eq. 1 does."""
    best, _, _, _, _ = postprocess(times)
    nv = len(times)
    pts = []
    for s in shapes:
        pts.append([best[s] / times[v][s] if _finite(times[v][s]) else 0.0 for v in range(nv)])
    return pts


def _pick_each(vectors, k, nv):
    """Best variant (largest component, lowest index on ties) of each
    representative vector, in order; a variant already taken is replaced by
    the vector's next best; at most k."""
    chosen = []
    for vec in vectors:
        order = sorted(range(nv), key=lambda v: (-vec[v], v))
        for v in order:
            if v not in chosen:
                chosen.append(v)
                break
    return chosen[:k]


def _pick_distinct(vectors, k, nv):
    """The sorted set of ``_pick_each``."""
    return tuple(sorted(_pick_each(vectors, k, nv)))


def kmeans_select(times, k, shapes, init, max_iter=100):
    """Lloyd's algorithm from the given initial centroids (indices into
    `shapes`): assign each point to its nearest centroid (squared Euclidean
    distance, lowest centroid on ties), move each centroid to the mean of its
    points (an empty cluster keeps its centroid), until no assignment
    changes.  Returns (kappa, assignment, iterations)."""
    pts = performance_vectors(times, shapes)
    nv = len(times)
    cents = [list(pts[i]) for i in init]
    assign = [-1] * len(pts)
    it = 0
    for it in range(1, max_iter + 1):
        new = []
        for p in pts:
            d = [sum((p[v] - c[v]) ** 2 for v in range(nv)) for c in cents]
            new.append(min(range(len(cents)), key=lambda j: (d[j], j)))
        changed = new != assign
        assign = new
        for j in range(len(cents)):
            mem = [pts[i] for i in range(len(pts)) if assign[i] == j]
            if mem:
                cents[j] = [sum(m[v] for m in mem) / len(mem) for v in range(nv)]
        if not changed:
            break
    return _pick_distinct(cents, k, nv), assign, it


# --- Sec. IV-C-3: decision tree with |kappa| leaves ----------------------------

def tree_model(times, k, shapes, features):
    """The tree of ``tree_select`` as a model: (kappa, leaf of each
    environment, nodes, leaf variants).  ``nodes[n]`` is (feature, threshold,
    left node, right node) for an internal node and (-1, 0.0, leaf index, -1)
    for a leaf; node 0 is the root and a split turns a leaf node into an
    internal node whose children are appended, left first.  ``leaf
    variants[l]`` is the variant leaf l contributed (its mean vector's best,
    or its next best if an earlier leaf took it)."""
    pts = performance_vectors(times, shapes)
    nv = len(times)

    def sse(idx):
        if not idx:
            return 0.0
        mean = [sum(pts[i][v] for i in idx) / len(idx) for v in range(nv)]
        return sum((pts[i][v] - mean[v]) ** 2 for i in idx for v in range(nv))

    def best_split(idx):
        base = sse(idx)
        best = None
        for f in range(len(features[0])):
            vals = sorted(set(features[i][f] for i in idx))
            for a, b in zip(vals, vals[1:]):
                thr = 0.5 * (a + b)
                left = [i for i in idx if features[i][f] <= thr]
                right = [i for i in idx if features[i][f] > thr]
                gain = base - sse(left) - sse(right)
                if best is None or gain > best[0] + 1e-12:
                    best = (gain, f, thr, left, right)
        return best

    leaves = [list(range(len(pts)))]
    leaf_node = [0]
    nodes = [None]
    while len(leaves) < k:
        cands = []
        for li, idx in enumerate(leaves):
            bs = best_split(idx)
            if bs is not None:
                cands.append((bs[0], li, bs))
        if not cands:
            break
        _, li, (gain, f, thr, left, right) = max(cands, key=lambda c: (c[0], -c[1]))
        n, a, b = leaf_node[li], len(nodes), len(nodes) + 1
        nodes[n] = (f, thr, a, b)
        nodes += [None, None]
        leaves[li:li + 1] = [left, right]
        leaf_node[li:li + 1] = [a, b]
    for li, n in enumerate(leaf_node):
        nodes[n] = (-1, 0.0, li, -1)
    reps = [[sum(pts[i][v] for i in idx) / len(idx) for v in range(nv)] for idx in leaves]
    leaf_of = [0] * len(pts)
    for li, idx in enumerate(leaves):
        for i in idx:
            leaf_of[i] = li
    each = _pick_each(reps, k, nv)
    return tuple(sorted(each)), leaf_of, nodes, each


def tree_route(nodes, x):
    """Leaf index of feature vector x: from the root, x[f] <= threshold goes
    to the left child."""
    n = 0
    while nodes[n][0] >= 0:
        f, thr, left, right = nodes[n]
        n = left if x[f] <= thr else right
    return nodes[n][2]


def tree_select(times, k, shapes, features):
    """Regression tree from environment features to performance vectors,
    grown best first to k leaves: repeatedly split the leaf whose best split
    lowers the summed squared error of the vectors most (thresholds halfway
    between consecutive distinct feature values; ties to the lower leaf,
    feature, threshold); each leaf's representative is the mean vector of
    its environments and contributes its best variant.
    Returns (kappa, leaf index of each environment)."""
    kappa, leaf_of, _, _ = tree_model(times, k, shapes, features)
    return kappa, leaf_of
