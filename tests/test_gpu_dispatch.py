"""GPU: the runtime's set dispatch (variant_set_load + variant_select) against
the oracle's rule on the committed set files, and sgemm() through a set
against the FP64 oracle.

The runtime tabulates the wave correction from the device it runs on; the
oracle is given the same inputs: the set file's training shapes and member
log-slowdowns, work-group counts of each member's launch (tiles times K
splits, ``space.Variant.work_groups``), and the device's compute-unit count.
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
FORMS = {"fp32": 0, "bf16x3": 1, "bf16x6": 2, "fp16s": 3}


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
    gt = [[variants[v].work_groups(*s) for v in members] for s in train]
    for q in _queries():
        gq = [variants[v].work_groups(*q) for v in members]
        want = pr.dispatch(train, members, cost, *q, gt, gq, cus)
        assert abi.variant_select_form(form, *q) == want, (fname, q)
    # Every training shape gets its own rule winner.
    for s, row in zip(train, cost):
        assert abi.variant_select_form(form, *s) == members[int(np.argmin(row))], (fname, s)


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
