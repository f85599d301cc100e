"""Variant-set files: where they live and how they are written.

A set file is the output of portability tuning (Sec. IV-B: a set kappa of
variants for a set of inputs) together with the online dispatch table
(Fig. 1: a picker that chooses one member per input).  Its format is read by
``variant_set_load`` in the runtime:

    fewfit-set 1
    arch gfx950
    codedir ../variants
    variant <id> <name> MWG NWG KWG MI WM WN SK VW LDS GM SG    (k lines)
    rule <M> <N> <K> <id> <c_1> ... <c_k>                    (training shapes)
    end

A rule names the training shape's winner and every member's log-slowdown
there (ln(t / best), "inf" where the member failed); the runtime uses these
to pick a member for shapes between training shapes.
"""
from __future__ import annotations

import os

from . import space

PKG = os.path.dirname(os.path.abspath(__file__))
SETS_DIR = os.path.join(PKG, "sets")
VARIANT_DIR = os.path.join(PKG, "variants")
FIXED_SET = os.path.join(SETS_DIR, "fixed_k1.txt")


def set_path(k: int, form: str = "fp32") -> str:
    if form == "fp32":
        return os.path.join(SETS_DIR, f"set_k{k}.txt")
    return os.path.join(SETS_DIR, f"set_{form}_k{k}.txt")


def default_set_path() -> str:
    """The tuned k=4 set when present, else the single fixed variant."""
    p = set_path(4)
    return p if os.path.exists(p) else FIXED_SET


def _fmt_cost(c):
    return "inf" if c == float("inf") else f"{c:.17g}"


def write_set_file(path, members, rules, arch="gfx950", codedir="../variants", comments=(), form="fp32"):
    """members: [(id, space.Variant)]; rules: [(M, N, K, winner_id, [cost per member])]."""
    ids = [vid for vid, _ in members]
    for r in rules:
        if r[3] not in ids or len(r[4]) != len(ids):
            raise ValueError(f"rule {r[:4]} does not match the set")
    lines = [f"# {c}" for c in comments]
    lines += ["fewfit-set 1", f"arch {arch}", f"codedir {codedir}"]
    if form != "fp32":
        lines.append(f"form {form}")
    lines += [f"variant {v.descriptor(vid)}" for vid, v in members]
    lines += [f"rule {M} {N} {K} {vid} " + " ".join(_fmt_cost(c) for c in cost)
              for (M, N, K, vid, cost) in rules]
    lines.append("end")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(tmp, path)


def write_fixed_set():
    """The one-variant set of the fixed 64x64 / K-step 16 kernel (id 0)."""
    write_set_file(FIXED_SET, [(0, space.DEFAULT)], [(256, 256, 256, 0, [0.0])],
                   comments=("single fixed variant: 64x64 tile, K-step 16",))
