"""Portability tuning on the measured table, set files, and evaluation.

Steps (Sec. IV, Sec. V-C, Sec. V-E), all arithmetic in libfewfit:

* post-processing: per-shape best (AutoTune, Sec. IV-A) and worst, slowdown
  and speedup of every entry (Sec. V-C, Table VI columns);
* PortabilityTune (Sec. IV-B): for k in {1, 2, 4, 8}, the set minimising
  Eq. 1 over the training shapes (exhaustive where feasible, greedy + swap
  otherwise);
* the dispatch table for the set file: the in-set winner of each training
  shape and every member's log-slowdown there; an unseen shape goes to the
  member with the smallest summed log-slowdown over its nearest training
  shapes, each moved to the unseen shape by the member's work-group wave
  efficiency on the device (``ptune_dispatch``);
* evaluation (Sec. V-E figures of merit): fraction of the per-shape best
  (1 / slowdown-over-best, geometric mean) on the held-out shapes as
  realised by the dispatch rule, and over all 27 shapes with a perfect
  in-set pick (how the paper evaluates, Fig. 1); geomean TFLOP/s.

Usage: python -m paper_2507_15277_amd.portability --table T.jsonl [--write-sets]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import abi, datagen, space, tuned
from .tune import load_rows, kernel_hash, current_hashes

PKG = os.path.dirname(os.path.abspath(__file__))
DATA_DIR = os.path.join(PKG, "data")
TABLE = os.path.join(DATA_DIR, "mi355x_table.jsonl")
# A second, independent FP32 table of the grid (another lease), for the
# robustness of the selection.
TABLE2 = os.path.join(DATA_DIR, "mi355x_table_run2.jsonl")
# Every form on the fresh shapes with lognormal operands (kept apart: only
# the accuracy-targeted set's generalisation report reads it).
TABLE_FRESH_LN = os.path.join(DATA_DIR, "mi355x_table_fresh_lognormal.jsonl")
KS = (1, 2, 4, 8)


def read_variants(directory=tuned.VARIANT_DIR):
    """{id: space.Variant} from the manifest."""
    out = {}
    with open(os.path.join(directory, "manifest.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                p = line.split()
                vals = [int(x) for x in p[2:]]
                out[int(p[0])] = space.Variant(*vals)
    return out


def matrix(rows, shapes, beta=0.0, nv=None, data="uniform", field="ms"):
    """Matrix x[v][s] of a row field (default the time in ms) for one input
    distribution; +inf where a variant failed or is missing."""
    nv = nv if nv is not None else 1 + max(r["variant"] for r in rows)
    idx = {tuple(s): j for j, s in enumerate(shapes)}
    t = np.full((nv, len(shapes)), np.inf)
    for r in rows:
        j = idx.get((r["M"], r["N"], r["K"]))
        if (j is None or r["beta"] != beta or r.get("status") != "ok"
                or r.get("data", "uniform") != data or r.get(field) is None):
            continue
        t[r["variant"], j] = r[field]
    return t


def geomean(xs):
    """Geometric mean; NaN for an empty sequence (e.g. no held-out shapes)."""
    xs = list(xs)
    if not xs:
        return math.nan
    return math.exp(sum(math.log(x) for x in xs) / len(xs))


def tflops(shape, ms):
    M, N, K = shape
    return 2.0 * M * N * K / ms / 1e9


# Compute units of the device the table was measured on (MI355X); the
# runtime queries the device it runs on.
DEVICE_CUS = 256
SO_EDGES = (1.0, 1.05, 1.1, 1.25, 1.5)   # S/O histogram bin edges (last bin open)
_VARIANTS = {}


def dispatch(train, kappa, costs, M, N, K):
    """The runtime's pick for (M, N, K): the neighbour vote with the wave
    correction for DEVICE_CUS compute units (``ptune_dispatch``)."""
    if not _VARIANTS:
        _VARIANTS.update(read_variants())
    gt = [[_VARIANTS[v].work_groups(*s) for v in kappa] for s in train]
    gq = [_VARIANTS[v].work_groups(M, N, K) for v in kappa]
    return abi.ptune_dispatch(train, kappa, costs, M, N, K, gt, gq, DEVICE_CUS)


def member_costs(t, kappa, train_idx):
    """ntrain x k matrix of ln(t[member][shape] / best[shape])."""
    best, _, _, _, _ = abi.ptune_postprocess(t)
    c = np.full((len(train_idx), len(kappa)), np.inf)
    for i, s in enumerate(train_idx):
        for j, v in enumerate(kappa):
            if np.isfinite(t[v, s]):
                c[i, j] = math.log(t[v, s] / best[s])
    return c


def evaluate(t, shapes, train_idx, kappa, extra=()):
    """Figures of merit of one set on the grid."""
    best, _, _, _, _ = abi.ptune_postprocess(t)
    train = [shapes[j] for j in train_idx]
    winners = abi.ptune_assign(t, kappa, train_idx)
    costs = member_costs(t, kappa, train_idx)
    held_idx = [j for j in range(len(shapes)) if j not in set(train_idx)]
    realised = {}
    for j, s in enumerate(shapes):
        realised[j] = dispatch(train, kappa, costs, *s)
    frac = lambda idx, pick: geomean(best[j] / t[pick(j), j] for j in idx)  # noqa: E731
    in_set = lambda j: min(kappa, key=lambda v: (t[v, j], v))  # noqa: E731
    # Per-shape slowdown of the dispatched member over the per-shape best
    # (the paper's S/O, Sec. V-E), over all shapes, as a histogram.
    so = [float(t[realised[j], j] / best[j]) for j in range(len(shapes))]
    edges = SO_EDGES + (math.inf,)
    hist = [sum(1 for x in so if lo <= x < hi) for lo, hi in zip(edges[:-1], edges[1:])]
    return {
        "kappa": list(kappa),
        "winners": winners,
        "so_max": max(so),
        "so_hist": {"edges": list(SO_EDGES), "counts": hist},
        "costs": costs.tolist(),
        "frac_heldout_realised": frac(held_idx, lambda j: realised[j]),
        "frac_heldout_inset": frac(held_idx, in_set),
        "frac_train": frac(train_idx, in_set),
        "frac_all_inset": frac(range(len(shapes)), in_set),
        "frac_all_realised": frac(range(len(shapes)), lambda j: realised[j]),
        "geomean_tflops_realised": geomean(tflops(s, t[realised[j], j]) for j, s in enumerate(shapes)),
        "per_shape": [{"M": s[0], "N": s[1], "K": s[2], "variant": int(realised[j]),
                       "tflops": tflops(s, t[realised[j], j]),
                       "best_tflops": tflops(s, best[j]), "frac": best[j] / t[realised[j], j],
                       "held_out": j not in set(train_idx)}
                      for j, s in enumerate(shapes)],
    }


def precision_report(rows, variants, write_sets=False, log=print):
    """Split-precision forms on the lognormal grid: per shape and form the
    fastest variant, its speedup over the fastest FP32 variant on the same
    inputs, and its errors against the FP64 reference; a k=4 set per form."""
    shapes = datagen.grid27()
    nv = len(variants)
    t = matrix(rows, shapes, 0.0, nv, data="lognormal")
    if not np.isfinite(t).any():
        return None
    en = matrix(rows, shapes, 0.0, nv, data="lognormal", field="err_norm")
    ec = matrix(rows, shapes, 0.0, nv, data="lognormal", field="err_comp")
    prec = np.array([variants[v].prec for v in range(nv)])
    train, _ = datagen.checkerboard_split(shapes)
    train_idx = [shapes.index(s) for s in train]
    out = {"forms": {}, "per_shape": []}
    best = {}
    for p in range(len(abi.FORM_NAMES)):
        tp = np.where((prec == p)[:, None], t, np.inf)
        if not np.isfinite(tp).any(axis=0).all():
            continue
        bid = [int(np.argmin(tp[:, j])) for j in range(len(shapes))]
        best[p] = bid
        form = abi.FORM_NAMES[p]
        errs = [float(en[bid[j], j]) for j in range(len(shapes))]
        comps = [float(ec[bid[j], j]) for j in range(len(shapes))]
        # The most accurate variant of the form as well (errors differ by
        # accumulation order).
        worst_all = float(np.max(np.where(np.isfinite(tp), en, 0.0)))
        rec = {"geomean_tflops_best": geomean(tflops(s, tp[bid[j], j]) for j, s in enumerate(shapes)),
               "max_err_norm_of_fastest": max(errs), "median_err_norm_of_fastest": float(np.median(errs)),
               "max_err_comp_of_fastest": max(comps), "max_err_norm_any_variant": worst_all}
        if p > 0:
            kappa, cost, _ = abi.ptune_select(tp, 4, shapes=train_idx, method=-1)
            ev = evaluate(tp, shapes, train_idx, kappa)
            rec.update(k4_kappa=list(kappa), k4_names=[variants[v].name for v in kappa],
                       k4_train_frac=1.0 / cost, k4_heldout_realised=ev["frac_heldout_realised"],
                       k4_geomean_tflops=ev["geomean_tflops_realised"])
            if write_sets:
                members = [(v, variants[v]) for v in kappa]
                rules = [(*shapes[j], w, ev["costs"][i])
                         for i, (j, w) in enumerate(zip(train_idx, ev["winners"]))]
                tuned.write_set_file(
                    tuned.set_path(4, form), members, rules, form=form,
                    comments=(f"PortabilityTune k=4 for the {form} form on the 14 checkerboard training "
                              f"shapes, lognormal operands",))
        out["forms"][form] = rec
        log(f"[precision] {form}: geomean {rec['geomean_tflops_best']:.2f} TFLOP/s (per-shape best), "
            f"normwise error of the fastest: median {rec['median_err_norm_of_fastest']:.2e} "
            f"max {rec['max_err_norm_of_fastest']:.2e}")
    for j, s in enumerate(shapes):
        rec = {"M": s[0], "N": s[1], "K": s[2]}
        for p, bid in best.items():
            form = abi.FORM_NAMES[p]
            rec[form] = {"variant": bid[j], "tflops": tflops(s, t[bid[j], j]),
                         "err_norm": float(en[bid[j], j]), "err_comp": float(ec[bid[j], j])}
            if p > 0 and 0 in best:
                rec[form]["speedup_vs_fp32"] = float(t[best[0][j], j] / t[bid[j], j])
        out["per_shape"].append(rec)
    if 0 in best:
        for p in best:
            if p > 0:
                form = abi.FORM_NAMES[p]
                out["forms"][form]["geomean_speedup_vs_fp32"] = geomean(
                    r[form]["speedup_vs_fp32"] for r in out["per_shape"])
    return out


ACCURACY_TARGET = 1e-6   # normwise error against FP64, the mixed set's target


def accuracy_report(rows, variants, target=ACCURACY_TARGET, write_sets=False, log=print):
    """Portability tuning with the precision form as one more variant
    parameter and an accuracy target as a constraint: on the lognormal grid a
    variant's time counts on a shape only where its measured normwise error
    meets the target (elsewhere +inf, as for a variant that fails the screen,
    Sec. V-C), then Eq. 1 selects k members from all forms together.  Beside
    it, the same selection within each form alone, and the unconstrained FP32
    set with the number of shapes where its dispatched member misses the
    target.  The k = 4 mixed set is written as the FF_FORM_MIXED set."""
    shapes = datagen.grid27()
    nv = len(variants)
    t = matrix(rows, shapes, 0.0, nv, data="lognormal")
    en = matrix(rows, shapes, 0.0, nv, data="lognormal", field="err_norm")
    if not np.isfinite(t).any():
        return None
    prec = np.array([variants[v].prec for v in range(nv)])
    ok = np.isfinite(en) & (en <= target)
    tt = np.where(ok, t, np.inf)
    train, _ = datagen.checkerboard_split(shapes)
    train_idx = [shapes.index(s) for s in train]
    out = {"target_err_norm": target, "data": "lognormal",
           "shapes_with_a_variant_meeting_target": {
               "any": int(ok.any(axis=0).sum()),
               **{abi.FORM_NAMES[p]: int(ok[prec == p].any(axis=0).sum()) for p in range(len(abi.FORM_NAMES))}},
           "per_shape_best_geomean_tflops": {}, "sets": {}, "single_form_k4": {}}

    def best_geomean(m):
        b = np.min(m, axis=0)
        return geomean(tflops(s, b[j]) for j, s in enumerate(shapes)) if np.isfinite(b).all() else None
    out["per_shape_best_geomean_tflops"]["mixed"] = best_geomean(tt)
    for p in range(len(abi.FORM_NAMES)):
        out["per_shape_best_geomean_tflops"][abi.FORM_NAMES[p]] = best_geomean(
            np.where((prec == p)[:, None], tt, np.inf))

    def realised_errors(ev):
        return [float(en[r["variant"], j]) for j, r in enumerate(ev["per_shape"])]
    for k in KS:
        kappa, cost, _ = abi.ptune_select(tt, k, shapes=train_idx, method=-1)
        ev = evaluate(tt, shapes, train_idx, kappa)
        errs = realised_errors(ev)
        out["sets"][str(k)] = {
            "kappa": list(kappa), "names": [variants[v].name for v in kappa],
            "forms": [abi.FORM_NAMES[prec[v]] for v in kappa], "train_frac": 1.0 / cost,
            "heldout_realised": ev["frac_heldout_realised"],
            "geomean_tflops_realised": ev["geomean_tflops_realised"],
            "realised_meeting_target": sum(1 for e in errs if e <= target),
            "realised_max_err_norm": max(errs),
            "per_shape": [{"M": r["M"], "N": r["N"], "K": r["K"], "variant": r["variant"],
                           "form": abi.FORM_NAMES[prec[r["variant"]]], "tflops": r["tflops"],
                           "err_norm": e} for r, e in zip(ev["per_shape"], errs)]}
        log(f"[accuracy] k={k} at err <= {target:g}: {list(kappa)} "
            f"({', '.join(out['sets'][str(k)]['forms'])}), geomean {ev['geomean_tflops_realised']:.2f} "
            f"TFLOP/s, held-out realised {ev['frac_heldout_realised']:.3f}")
        if write_sets and k == 4:
            members = [(v, variants[v]) for v in kappa]
            rules = [(*shapes[j], w, ev["costs"][i])
                     for i, (j, w) in enumerate(zip(train_idx, ev["winners"]))]
            tuned.write_set_file(
                tuned.set_path(4, "mixed"), members, rules, form="mixed",
                comments=(f"PortabilityTune k=4 over every form's variants on the 14 checkerboard training "
                          f"shapes, lognormal operands, counting a variant only where its normwise error "
                          f"is at most {target:g}",))
    for p in range(len(abi.FORM_NAMES)):
        tp = np.where((prec == p)[:, None], tt, np.inf)
        if not np.isfinite(tp).any(axis=0).all():
            continue
        kappa, cost, _ = abi.ptune_select(tp, 4, shapes=train_idx, method=-1)
        ev = evaluate(tp, shapes, train_idx, kappa)
        out["single_form_k4"][abi.FORM_NAMES[p]] = {
            "kappa": list(kappa), "geomean_tflops_realised": ev["geomean_tflops_realised"],
            "heldout_realised": ev["frac_heldout_realised"]}
    # The unconstrained FP32 set (its timing on these inputs, no target).
    t32 = np.where((prec == 0)[:, None], t, np.inf)
    kappa, _, _ = abi.ptune_select(t32, 4, shapes=train_idx, method=-1)
    ev = evaluate(t32, shapes, train_idx, kappa)
    errs = realised_errors(ev)
    out["fp32_k4_unconstrained"] = {"kappa": list(kappa), "geomean_tflops_realised": ev["geomean_tflops_realised"],
                                    "realised_meeting_target": sum(1 for e in errs if e <= target),
                                    "realised_max_err_norm": max(errs)}
    return out


def accuracy_fresh_report(rows, variants, target=ACCURACY_TARGET, log=print):
    """The committed mixed set and the FP32 k = 4 set, frozen, on the fresh
    shapes with lognormal operands (timed after the sets were chosen): each
    shape dispatched by the runtime's rule, its member's time and measured
    normwise error against the fastest variant of any form that meets the
    target on that shape."""
    shapes = datagen.fresh_shapes()
    nv = len(variants)
    t = matrix(rows, shapes, 0.0, nv, data="lognormal")
    en = matrix(rows, shapes, 0.0, nv, data="lognormal", field="err_norm")
    if not np.isfinite(t).any(axis=0).all():
        return None
    tt = np.where(np.isfinite(en) & (en <= target), t, np.inf)
    best = np.min(tt, axis=0)
    n_grid = 37
    out = {"target_err_norm": target, "n_shapes": len(shapes), "n_paper_grid": n_grid,
           "per_shape_best_geomean_tflops": geomean(tflops(s, best[j]) for j, s in enumerate(shapes)), "sets": {}}
    for label, path in (("mixed_k4", tuned.set_path(4, "mixed")), ("fp32_k4", tuned.set_path(4))):
        members, train, cost = read_set(path)
        picks = [dispatch(train, members, cost, *s) for s in shapes]
        ts = [float(t[p, j]) for j, p in enumerate(picks)]
        es = [float(en[p, j]) for j, p in enumerate(picks)]
        ok = [j for j in range(len(shapes)) if np.isfinite(ts[j])]
        met = [j for j in ok if es[j] <= target]
        # Speed as a fraction of the fastest variant meeting the target, on
        # the shapes where the dispatched member meets it too.
        frac = lambda idx: geomean(best[j] / ts[j] for j in idx if np.isfinite(best[j]))  # noqa: E731
        out["sets"][label] = {
            "geomean_tflops_realised": geomean(tflops(shapes[j], ts[j]) for j in ok),
            "frac_of_best_meeting_target": frac(met),
            "frac_paper_grid": frac([j for j in met if j < n_grid]),
            "frac_random": frac([j for j in met if j >= n_grid]),
            "meeting_target": len(met), "timed": len(ok),
            "max_err_norm": max(es[j] for j in ok),
            "missed": [{"M": shapes[j][0], "N": shapes[j][1], "K": shapes[j][2], "err_norm": es[j],
                        "form": abi.FORM_NAMES[variants[picks[j]].prec]} for j in ok if es[j] > target]}
        log(f"[accuracy fresh] {label}: geomean {out['sets'][label]['geomean_tflops_realised']:.1f} TFLOP/s, "
            f"{out['sets'][label]['meeting_target']}/{len(ok)} shapes meet {target:g}")
    return out


def accuracy_training_report(rows, variants, target=ACCURACY_TARGET, log=print):
    """Whether more training shapes help the accuracy-targeted selection on
    unseen ones: the constrained selection trained on the 14 checkerboard
    grid shapes and on the paper's whole 64-shape {256, 512, 1024, 4096}^3
    grid (the 27 grid shapes plus the 37 fresh ones off it), each scored by
    dispatch on the 20 random fresh shapes, which neither saw.  ``rows``
    must hold the lognormal rows of both the grid and the fresh shapes."""
    grid, fresh = datagen.grid27(), datagen.fresh_shapes()
    shapes = list(grid) + list(fresh)
    nv = len(variants)
    t = matrix(rows, shapes, 0.0, nv, data="lognormal")
    en = matrix(rows, shapes, 0.0, nv, data="lognormal", field="err_norm")
    if not np.isfinite(t).any(axis=0).all():
        return None
    tt = np.where(np.isfinite(en) & (en <= target), t, np.inf)
    best = np.min(tt, axis=0)
    train14, _ = datagen.checkerboard_split(grid)
    trainings = {"grid14": [shapes.index(s) for s in train14],
                 "paper_grid64": list(range(len(grid) + 37))}
    held = list(range(len(grid) + 37, len(shapes)))
    out = {"target_err_norm": target, "held_out": [list(shapes[j]) for j in held], "sets": {}}
    for label, tr in trainings.items():
        train = [shapes[j] for j in tr]
        for k in (4, 8):
            kappa, cost, _ = abi.ptune_select(tt, k, shapes=tr, method=-1)
            costs = member_costs(tt, kappa, tr)
            picks = {j: dispatch(train, kappa, costs, *shapes[j]) for j in held}
            rec = {"kappa": list(kappa), "forms": [abi.FORM_NAMES[variants[v].prec] for v in kappa],
                   "train_frac": 1.0 / cost,
                   "heldout_frac": geomean(best[j] / t[picks[j], j] for j in held),
                   "heldout_geomean_tflops": geomean(tflops(shapes[j], t[picks[j], j]) for j in held),
                   "heldout_meeting_target": sum(1 for j in held if en[picks[j], j] <= target)}
            out["sets"][f"{label}_k{k}"] = rec
            log(f"[accuracy training] {label} k={k}: held-out fraction {rec['heldout_frac']:.3f}, "
                f"{rec['heldout_meeting_target']}/{len(held)} meet {target:g}")
    return out


SWEEP_TARGETS = (3e-4, 1e-5, 1e-6, 5e-7)


def accuracy_sweep(rows, variants, targets=SWEEP_TARGETS, log=print):
    """The accuracy target against speed: for each target the per-shape best
    geomean over every form's variants that meet it, and the k = 4 set chosen
    under it (its forms and realised geomean)."""
    out = []
    for tau in targets:
        r = accuracy_report(rows, variants, target=tau, log=lambda *_: None)
        if r is None:
            return None
        s4 = r["sets"]["4"]
        out.append({"target_err_norm": tau, "per_shape_best_geomean_tflops": r["per_shape_best_geomean_tflops"]["mixed"],
                    "k4_kappa": s4["kappa"], "k4_forms": s4["forms"],
                    "k4_geomean_tflops_realised": s4["geomean_tflops_realised"],
                    "k4_realised_meeting_target": s4["realised_meeting_target"],
                    "k4_realised_max_err_norm": s4["realised_max_err_norm"]})
        log(f"[accuracy sweep] err <= {tau:g}: best {out[-1]['per_shape_best_geomean_tflops']:.1f}, k=4 "
            f"{s4['geomean_tflops_realised']:.1f} TFLOP/s ({', '.join(s4['forms'])})")
    return out


def read_set(path):
    """(members, training shapes, ntrain x k member log-slowdowns) of a set file."""
    members, train, cost = [], [], []
    with open(path) as f:
        for line in f:
            p = line.split("#")[0].split()
            if not p:
                continue
            if p[0] == "variant":
                members.append(int(p[1]))
            elif p[0] == "rule":
                train.append(tuple(int(x) for x in p[1:4]))
                cost.append([float(x) for x in p[5:]])
    return members, train, np.array(cost)


def fresh_report(rows, variants, log=print):
    """Generalisation to shapes that chose nothing (Sec. V-H, V-I, Fig. 1):
    the committed sets and their dispatch rule, frozen, on the 37 shapes of
    the paper's {256, 512, 1024, 4096}^3 grid off the tuning grid and on
    seeded log-uniform shapes in [128, 8192].  Per set: the fraction of the
    per-shape best realised through dispatch and with a perfect in-set pick,
    and the slowdown over the per-shape best (S/O) as a histogram."""
    shapes = datagen.fresh_shapes()
    n_paper = len(shapes) - 20
    nv = len(variants)
    t = matrix(rows, shapes, 0.0, nv)
    fp32 = np.array([variants[v].prec == 0 for v in range(nv)])
    t[~fp32, :] = np.inf
    cols = [j for j in range(len(shapes)) if np.isfinite(t[:, j]).any()]
    if len(cols) < len(shapes):
        return None
    best = t.min(axis=0)
    out = {"shapes": [list(s) for s in shapes], "n_paper_grid": n_paper,
           "geomean_tflops_best": geomean(tflops(s, best[j]) for j, s in enumerate(shapes)), "sets": {}}
    edges = SO_EDGES + (math.inf,)
    labels = [("fixed", tuned.FIXED_SET)] + \
        [(f"k{k}", tuned.set_path(k)) for k in KS]
    for label, path in labels:
        members, train, cost = read_set(path)
        picks = [dispatch(train, members, cost, *s) for s in shapes]
        real = [float(best[j] / t[picks[j], j]) for j in range(len(shapes))]
        inset = [float(best[j] / min(t[v, j] for v in members)) for j in range(len(shapes))]
        so = [1.0 / x for x in real]
        rec = {"members": members,
               "frac_realised": geomean(real), "frac_inset": geomean(inset),
               "frac_realised_paper_grid": geomean(real[:n_paper]),
               "frac_realised_random": geomean(real[n_paper:]),
               "frac_inset_paper_grid": geomean(inset[:n_paper]),
               "frac_inset_random": geomean(inset[n_paper:]),
               "geomean_tflops_realised": geomean(tflops(s, t[picks[j], j]) for j, s in enumerate(shapes)),
               "so_max": max(so),
               "so_hist": {"edges": list(SO_EDGES),
                           "counts": [sum(1 for x in so if lo <= x < hi) for lo, hi in zip(edges[:-1], edges[1:])]},
               "per_shape": [{"M": s[0], "N": s[1], "K": s[2], "variant": int(picks[j]),
                              "frac": real[j], "inset_frac": inset[j]} for j, s in enumerate(shapes)]}
        out["sets"][label] = rec
        log(f"[fresh] {label}: realised {rec['frac_realised']:.4f} (paper grid {rec['frac_realised_paper_grid']:.4f}, "
            f"random {rec['frac_realised_random']:.4f}), in-set {rec['frac_inset']:.4f}, max S/O {rec['so_max']:.2f}")
    return out


def ragged_report(rows, variants, log=print):
    """A selection that sees unaligned inputs.  The ragged grid (the 27 grid
    shapes moved off every multiple of 4, so every variant runs its
    scalar-load kernel) is timed like the grid; sets are chosen on the 14
    aligned training shapes (as committed) and on those plus their 14 ragged
    counterparts, and each is scored with a perfect in-set pick (Fig. 1's
    evaluation) on the held-out aligned and ragged shapes and on the fresh
    shapes: how much of the loss on ragged inputs is the selection's."""
    grid, rag, fresh = datagen.grid27(), datagen.ragged_grid(), datagen.fresh_shapes()
    shapes = grid + rag + fresh
    nv = len(variants)
    t = matrix(rows, shapes, 0.0, nv)
    t[np.array([variants[v].prec != 0 for v in range(nv)]), :] = np.inf
    if not np.isfinite(t).any(axis=0).all():
        return None
    best = t.min(axis=0)
    train, _ = datagen.checkerboard_split(grid)
    tr_g = [grid.index(s) for s in train]
    tr_r = [len(grid) + j for j in tr_g]
    ho_g = [j for j in range(len(grid)) if j not in tr_g]
    ho_r = [len(grid) + j for j in ho_g]
    n_paper = len(fresh) - 20
    fr_p = list(range(2 * len(grid), 2 * len(grid) + n_paper))
    fr_r = list(range(2 * len(grid) + n_paper, len(shapes)))

    def inset(kap, idx):
        return geomean(best[j] / min(t[v, j] for v in kap) for j in idx)

    out = {"ragged_best_geomean_tflops": geomean(tflops(s, best[len(grid) + j]) for j, s in enumerate(rag)),
           "aligned_best_geomean_tflops": geomean(tflops(s, best[j]) for j, s in enumerate(grid)), "sets": {}}
    for k in KS:
        rec = {}
        for label, tr in (("aligned_training", tr_g), ("aligned_and_ragged_training", tr_g + tr_r)):
            kap, _, _ = abi.ptune_select(t, k, shapes=tr, method=-1)
            rec[label] = {"kappa": list(kap), "heldout_aligned": inset(kap, ho_g), "heldout_ragged": inset(kap, ho_r),
                          "fresh_paper_grid": inset(kap, fr_p), "fresh_ragged": inset(kap, fr_r)}
        out["sets"][str(k)] = rec
        a, m = rec["aligned_training"], rec["aligned_and_ragged_training"]
        log(f"[ragged] k={k}: aligned training: held-out aligned {a['heldout_aligned']:.3f} ragged "
            f"{a['heldout_ragged']:.3f}, fresh ragged {a['fresh_ragged']:.3f}; with ragged training: "
            f"{m['heldout_aligned']:.3f} / {m['heldout_ragged']:.3f} / {m['fresh_ragged']:.3f}")
    return out


def robustness_report(rows, rows2, variants, log=print):
    """How much the selection rests on one table build (Sec. V-C, V-E): a
    second FP32 table of the same grid, timed independently on another
    lease, against the first.  Per shape the spread of the per-shape best;
    per k the sets chosen from each table, their overlap, each set's
    fraction of the per-shape best on the other table, and the sets chosen
    from mean instead of median times; the shader clock seen while timing."""
    shapes = datagen.grid27()
    nv = len(variants)
    t1 = matrix(rows, shapes, 0.0, nv)
    t2 = matrix(rows2, shapes, 0.0, nv)
    if not (np.isfinite(t2).any(axis=0).all() and np.isfinite(t1).any(axis=0).all()):
        return None
    tm = matrix(rows, shapes, 0.0, nv, field="ms_mean")
    train, _ = datagen.checkerboard_split(shapes)
    train_idx = [shapes.index(s) for s in train]
    b1, b2 = t1.min(axis=0), t2.min(axis=0)
    spread = np.abs(b2 / b1 - 1.0)
    out = {"per_shape_best_rel_diff_median": float(np.median(spread)),
           "per_shape_best_rel_diff_max": float(np.max(spread)),
           "geomean_tflops_best": [geomean(tflops(s, b1[j]) for j, s in enumerate(shapes)),
                                   geomean(tflops(s, b2[j]) for j, s in enumerate(shapes))],
           "same_per_shape_winner": int(sum(int(np.argmin(t1[:, j])) == int(np.argmin(t2[:, j]))
                                            for j in range(len(shapes)))),
           "sets": {}}
    for k in KS:
        k1, c1, _ = abi.ptune_select(t1, k, shapes=train_idx, method=-1)
        k2, c2, _ = abi.ptune_select(t2, k, shapes=train_idx, method=-1)
        km, _, _ = abi.ptune_select(tm, k, shapes=train_idx, method=-1)
        rec = {"kappa_run1": list(k1), "kappa_run2": list(k2), "overlap": len(set(k1) & set(k2)),
               "train_frac_run1": 1.0 / c1, "train_frac_run2": 1.0 / c2,
               "run1_set_on_run2": 1.0 / abi.ptune_cost(t2, k1, train_idx),
               "run2_set_on_run1": 1.0 / abi.ptune_cost(t1, k2, train_idx),
               "all27_run1_set_on_run2": 1.0 / abi.ptune_cost(t2, k1),
               "kappa_mean_selection": list(km), "mean_vs_median_overlap": len(set(km) & set(k1)),
               "mean_set_train_frac_median_times": 1.0 / abi.ptune_cost(t1, km, train_idx)}
        out["sets"][str(k)] = rec
        log(f"[robust] k={k}: run1 {list(k1)} run2 {list(k2)} overlap {rec['overlap']}; run1 set on run2 "
            f"{rec['run1_set_on_run2']:.4f} (own {rec['train_frac_run2']:.4f}); mean-selected {list(km)}")
    for name, rr in (("run1", rows), ("run2", rows2)):
        clk = [r["sclk_mhz"] for r in rr if r.get("sclk_mhz") and r.get("status") == "ok"
               and (r["M"], r["N"], r["K"]) in set(shapes)]
        if clk:
            out[f"sclk_mhz_{name}"] = {"median": float(np.median(clk)), "min": float(np.min(clk)),
                                       "max": float(np.max(clk)), "samples": len(clk)}
    return out


def selector_comparison(t, shapes, train_idx, runs=30, log=print):
    """PortabilityTune (exact search) against the paper's two pruning
    implementations (Sec. IV-C-2, IV-C-3), on the training shapes, for each
    k: fraction of per-shape best on the training shapes and realised on the
    held-out shapes (all sets dispatched by the same rule), and selection
    wall time.  k-means runs 30 times from seeded initial centroids (the
    paper reports the mean and a 95% interval over 30 runs, Sec. V-E)."""
    held_idx = [j for j in range(len(shapes)) if j not in set(train_idx)]
    feats = [[math.log2(x) for x in shapes[j]] for j in train_idx]
    out = {}
    for k in KS:
        rec = {}
        t0 = time.perf_counter()
        kap, cost, _ = abi.ptune_select(t, k, shapes=train_idx, method=-1)
        dt = time.perf_counter() - t0
        ev = evaluate(t, shapes, train_idx, kap)
        rec["portability_tune"] = {"kappa": list(kap), "train_frac": 1.0 / cost,
                                   "heldout_realised": ev["frac_heldout_realised"], "seconds": dt}
        fr_tr, fr_ho, secs = [], [], []
        for r in range(runs):
            rng = np.random.default_rng([9, k, r])
            init = sorted(rng.choice(len(train_idx), min(k, len(train_idx)), replace=False).tolist())
            t0 = time.perf_counter()
            kk, _, _ = abi.ptune_kmeans(t, len(init), train_idx, init)
            secs.append(time.perf_counter() - t0)
            fr_tr.append(1.0 / abi.ptune_cost(t, kk, train_idx))
            fr_ho.append(evaluate(t, shapes, train_idx, kk)["frac_heldout_realised"])
        ci = lambda x: 1.96 * float(np.std(x, ddof=1)) / math.sqrt(len(x))  # noqa: E731
        rec["kmeans"] = {"train_frac_mean": float(np.mean(fr_tr)), "train_frac_ci95": ci(fr_tr),
                         "train_frac_max": float(np.max(fr_tr)),
                         "heldout_realised_mean": float(np.mean(fr_ho)), "heldout_realised_ci95": ci(fr_ho),
                         "seconds_mean": float(np.mean(secs)), "runs": runs}
        t0 = time.perf_counter()
        kt, _, nf, nt, nc, lv = abi.ptune_tree(t, k, train_idx, feats, model=True)
        dt = time.perf_counter() - t0
        # The tree as its own runtime classifier: an unseen shape goes down
        # the splits (log2 M, N, K) to a leaf and runs that leaf's variant.
        routed = [lv[abi.ptune_tree_route(nf, nt, nc, [math.log2(x) for x in shapes[j]])]
                  for j in held_idx]
        best, _, _, _, _ = abi.ptune_postprocess(t)
        rec["decision_tree"] = {"kappa": list(kt), "train_frac": 1.0 / abi.ptune_cost(t, kt, train_idx),
                                "heldout_realised": evaluate(t, shapes, train_idx, kt)["frac_heldout_realised"],
                                "heldout_routed": geomean(best[j] / t[v, j] for j, v in zip(held_idx, routed)),
                                "seconds": dt}
        out[str(k)] = rec
        log(f"[selectors] k={k}: PortabilityTune {rec['portability_tune']['train_frac']:.4f}, "
            f"k-means {rec['kmeans']['train_frac_mean']:.4f} +- {rec['kmeans']['train_frac_ci95']:.4f}, "
            f"tree {rec['decision_tree']['train_frac']:.4f} (training shapes); held-out "
            f"{rec['portability_tune']['heldout_realised']:.4f} / "
            f"{rec['decision_tree']['heldout_realised']:.4f} (vote) / "
            f"{rec['decision_tree']['heldout_routed']:.4f} (tree routes)")
    return out


def fleet_comparison(t, shapes, log=print):
    """Eq. 2 with one device: a task runs every grid shape once (weight 1,
    as the paper's fleet task runs every known input once).  Sets chosen for
    the total time of a task against sets chosen by Eq. 1, both with a
    perfect in-set pick, and against the per-shape best (the lower bound)."""
    idx = list(range(len(shapes)))
    w = np.ones(len(shapes))
    best, _, _, _, _ = abi.ptune_postprocess(t)
    floor = float(np.sum(best))
    out = {"task_ms_per_shape_best": floor}
    for k in KS:
        kt, tot, _ = abi.ptune_select_total(t, k, idx, w, method=-1)
        ke, _, _ = abi.ptune_select(t, k, method=-1)
        tot_e = float(sum(min(t[v, j] for v in ke) for j in idx))
        out[str(k)] = {"total_kappa": list(kt), "task_ms": tot, "rate_vs_best": floor / tot,
                       "geomean_frac": 1.0 / abi.ptune_cost(t, kt),
                       "eq1_kappa": list(ke), "eq1_task_ms": tot_e, "eq1_rate_vs_best": floor / tot_e,
                       "eq1_geomean_frac": 1.0 / abi.ptune_cost(t, ke)}
        log(f"[fleet] k={k}: task time {tot:.3f} ms (Eq. 2 set) vs {tot_e:.3f} ms (Eq. 1 set), "
            f"best {floor:.3f} ms; geomean fraction {out[str(k)]['geomean_frac']:.3f} vs "
            f"{out[str(k)]['eq1_geomean_frac']:.3f}")
    return out


def run(table=TABLE, write_sets=False, splits=5, log=print):
    rows = load_rows(table, current_hashes())
    if not rows:
        raise RuntimeError(f"no rows for the current kernel source in {table}")
    variants = read_variants()
    nv = len(variants)
    shapes = datagen.grid27()
    t = matrix(rows, shapes, 0.0, nv)
    train, held = datagen.checkerboard_split(shapes)
    train_idx = [shapes.index(s) for s in train]
    best, worst, best_id, slow, speed = abi.ptune_postprocess(t)
    report = {"device": rows[0].get("device"), "n_variants": nv,
              "n_rows": len(rows), "kernel_build": kernel_hash(),
              "per_shape_best": [{"M": s[0], "N": s[1], "K": s[2], "variant": int(best_id[j]),
                                  "name": variants[int(best_id[j])].name,
                                  "tflops": tflops(s, best[j])} for j, s in enumerate(shapes)],
              "geomean_tflops_best": geomean(tflops(s, best[j]) for j, s in enumerate(shapes)),
              "distinct_winners": len(set(int(b) for b in best_id)),
              "sets": {}}
    # Middle 50% of variant slowdowns per shape (the paper quotes this band
    # to describe how sensitive a device is to tuning, Sec. IV-D-1).
    q25, q75 = [], []
    for j in range(len(shapes)):
        col = slow[:, j][np.isfinite(slow[:, j])]
        q25.append(float(np.percentile(col, 25)))
        q75.append(float(np.percentile(col, 75)))
    report["slowdown_middle50_median"] = [float(np.median(q25)), float(np.median(q75))]
    # The fixed single variant (id 0) as the one-variant baseline.
    report["fixed_variant"] = evaluate(t, shapes, train_idx, (0,))
    for k in KS:
        t0 = time.perf_counter()
        kappa, cost, evals = abi.ptune_select(t, k, shapes=train_idx, method=-1)
        dt = time.perf_counter() - t0
        ev = evaluate(t, shapes, train_idx, kappa)
        ev.update(train_cost=cost, evals=int(evals), select_seconds=dt,
                  names=[variants[v].name for v in kappa])
        report["sets"][str(k)] = ev
        log(f"[select] k={k}: kappa={list(kappa)} train F={1 / cost:.4f} held-out realised "
            f"F={ev['frac_heldout_realised']:.4f} all in-set F={ev['frac_all_inset']:.4f} "
            f"geomean {ev['geomean_tflops_realised']:.2f} TFLOP/s ({evals} subsets, {dt:.2f} s)")
        if write_sets:
            members = [(v, variants[v]) for v in kappa]
            rules = [(*shapes[j], w, ev["costs"][i])
                     for i, (j, w) in enumerate(zip(train_idx, ev["winners"]))]
            tuned.write_set_file(
                tuned.set_path(k), members, rules,
                comments=(f"PortabilityTune k={k} on the 14 checkerboard training shapes of the "
                          f"{{256,1024,4096}}^3 grid, MI355X table {os.path.basename(table)}",
                          f"train fraction of per-shape best {1 / cost:.4f}; held-out realised "
                          f"{ev['frac_heldout_realised']:.4f}"))
    # Robustness band: seeded random 14/13 splits.
    band = {str(k): [] for k in KS}
    for seed in range(splits):
        tr, _ = datagen.random_split(seed, 14, shapes)
        tri = [shapes.index(s) for s in tr]
        for k in KS:
            kappa, cost, _ = abi.ptune_select(t, k, shapes=tri, method=-1)
            band[str(k)].append(evaluate(t, shapes, tri, kappa)["frac_heldout_realised"])
    report["random_split_heldout_realised"] = band
    # Shapes from the paper's default-kernel example, two of them off the grid.
    extra_shapes = [(512, 4096, 4096), (4096, 4096, 512), (1024, 1024, 4096), (4096, 1024, 4096)]
    te = matrix(rows, extra_shapes, 0.0, nv)
    if np.isfinite(te).any(axis=0).all():
        be, _, _, _, _ = abi.ptune_postprocess(te)
        ex = {"fixed_variant": [float(be[j] / te[0, j]) for j in range(len(extra_shapes))]}
        for k in KS:
            ev = report["sets"][str(k)]
            trs = [shapes[j] for j in train_idx]
            picks = [dispatch(trs, ev["kappa"], ev["costs"], *s) for s in extra_shapes]
            ex[f"k{k}"] = [float(be[j] / te[p, j]) for j, p in enumerate(picks)]
        report["default_example_shapes"] = {"shapes": extra_shapes, "frac_of_best": ex}
    # Square sweep (beta 0 and 0.5): per-shape best and whether beta moves it.
    sq = datagen.square_shapes()
    sq_out = []
    for beta in (0.0, 0.5):
        ts = matrix(rows, sq, beta, nv)
        if not np.isfinite(ts).any():
            continue
        b, _, bid, sl, _ = abi.ptune_postprocess(ts)
        for j, s in enumerate(sq):
            col = sl[:, j][np.isfinite(sl[:, j])]
            sq_out.append({"M": s[0], "beta": beta, "best_variant": int(bid[j]),
                           "best_tflops": tflops(s, b[j]),
                           "fixed_variant_tflops": tflops(s, ts[0, j]),
                           "slowdown_q25": float(np.percentile(col, 25)),
                           "slowdown_q75": float(np.percentile(col, 75)),
                           "n_ok": int(np.isfinite(ts[:, j]).sum())})
    report["square_sweep"] = sq_out
    report["selectors"] = selector_comparison(t, shapes, train_idx, log=log)
    report["fleet"] = fleet_comparison(t, shapes, log=log)
    report["precision"] = precision_report(rows, variants, write_sets, log)
    report["accuracy"] = accuracy_report(rows, variants, write_sets=write_sets, log=log)
    if report["accuracy"] is not None:
        report["accuracy"]["sweep"] = accuracy_sweep(rows, variants, log=log)
        if os.path.exists(TABLE_FRESH_LN):
            rows_fl = load_rows(TABLE_FRESH_LN, current_hashes())
            report["accuracy"]["fresh"] = accuracy_fresh_report(rows_fl, variants, log=log)
            report["accuracy"]["training"] = accuracy_training_report(rows + rows_fl, variants, log=log)
    report["fresh"] = fresh_report(rows, variants, log)
    report["ragged"] = ragged_report(rows, variants, log)
    if os.path.exists(TABLE2):
        report["robustness"] = robustness_report(rows, load_rows(TABLE2, {kernel_hash()}), variants, log)
    if write_sets:
        tuned.write_fixed_set()
    report["screen"] = {
        "ok": sum(1 for r in rows if r.get("status") == "ok"),
        "wrong": sum(1 for r in rows if r.get("status") == "wrong"),
        "launch_fail": sum(1 for r in rows if r.get("status") == "launch_fail"),
        "max_err_ratio": max((r.get("err_ratio") or 0.0) for r in rows if r.get("status") == "ok"),
    }
    return report


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--table", default=TABLE)
    ap.add_argument("--write-sets", action="store_true")
    ap.add_argument("--report", default=os.path.join(DATA_DIR, "mi355x_report.json"))
    args = ap.parse_args(argv)
    rep = run(args.table, write_sets=args.write_sets, log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(args.report), exist_ok=True)
    with open(args.report, "w") as f:
        json.dump(rep, f, indent=1)
    print(f"geomean TFLOP/s of per-shape best: {rep['geomean_tflops_best']:.2f}; "
          f"distinct winners {rep['distinct_winners']}; screen {rep['screen']}")


if __name__ == "__main__":
    main()
