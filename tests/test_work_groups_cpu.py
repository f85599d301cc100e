"""Work-group counts of a variant's launch, worked out by hand.

The dispatch's wave correction (the runtime's variant_select and the
oracle's dispatch rule) reads, for every set member, the number of
work-groups its GEMM launch holds on a shape: the tiles of C times the
number of work-groups sharing one tile's K range.  Each case below states
that count from the variant's parameters with the arithmetic spelled out,
so a mistake in ``space.Variant.work_groups`` (a dropped ceiling, the split
clamp, K padding of the pre-split forms, the workspace limit) fails here;
the GPU dispatch test compares the runtime's own count
(``variant_work_groups``) with the same hand values.
"""
import pytest

from paper_2507_15277_amd import space

MiB = 1 << 20


def fp32(mwg, nwg, kwg, sg=1):
    return space.Variant(mwg, nwg, kwg, 32, 2, 2, 1, 4, 1, 8, sg, 0, 1)


def presplit(mwg, nwg, kwg, sg=1, prec=1):
    return space.Variant(mwg, nwg, kwg, 32, 2, 2, 1, 4, 2, 8, sg, prec, 1)


# (variant, (M, N, K), expected work-groups, how the count arises)
CASES = [
    (fp32(64, 128, 32), (4096, 4096, 4096), 64 * 32, "64 tile rows x 32 tile columns, no split"),
    (fp32(64, 64, 16), (300, 500, 700), 5 * 8, "ceil(300/64)=5 x ceil(500/64)=8"),
    (fp32(64, 64, 16), (1, 1, 1), 1, "one partial tile"),
    (fp32(64, 64, 16), (0, 64, 64), 0, "empty product launches nothing"),
    (fp32(64, 64, 16), (64, 0, 64), 0, "empty product launches nothing"),
    # SG = 4 on 256 x 256 x 4096 with 32 x 32 tiles and 32-deep slabs:
    # 8 x 8 tiles; 128 slabs; min(4, 128, 512 slices fit) = 4 splits of 32.
    (fp32(32, 32, 32, sg=4), (256, 256, 4096), 64 * 4, "64 tiles x 4 splits"),
    # SG = 8, K = 640 with 64-deep slabs: 10 slabs; 8 splits would hold
    # ceil(10/8) = 2 slabs each, so only ceil(10/2) = 5 splits are non-empty.
    (fp32(64, 64, 64, sg=8), (256, 256, 640), 16 * 5, "16 tiles x 5 non-empty splits"),
    # More splits allowed than slabs: K = 96 in 32-deep slabs is 3 slabs.
    (fp32(32, 32, 32, sg=16), (128, 128, 96), 16 * 3, "16 tiles x 3 single-slab splits"),
    # One slab: never split.
    (fp32(32, 32, 32, sg=16), (128, 128, 32), 16, "a single slab is not split"),
    # Workspace clamp: a 4096 x 4096 slice is 64 MiB, two fit in 128 MiB.
    (fp32(128, 128, 16, sg=8), (4096, 4096, 1024), 32 * 32 * 2, "1024 tiles x 2 slices that fit"),
    # 8192 x 8192 slices are 256 MiB: none fit, so no split.
    (fp32(128, 128, 16, sg=8), (8192, 8192, 1024), 64 * 64, "no slice fits: unsplit"),
    # 4096 x 2048: 32 MiB slices, 4 fit; SG 8 clamps to 4.
    (fp32(128, 128, 16, sg=8), (4096, 2048, 4096), 32 * 16 * 4, "512 tiles x 4 slices"),
    # Pre-split forms run over K padded to 64: K = 100 -> 128 -> two 64-deep
    # slabs, so SG 4 gives 2 splits.
    (presplit(64, 64, 64, sg=4), (64, 64, 100), 1 * 2, "K padded to 128: 2 slabs, 2 splits"),
    (presplit(128, 128, 64), (4096, 256, 256), 32 * 2, "32 x 2 tiles, no split"),
    # K = 64 exactly: one slab after padding, not split.
    (presplit(64, 64, 64, sg=4), (64, 64, 64), 1, "one padded slab is not split"),
]


@pytest.mark.parametrize("v,shape,want,why", CASES, ids=[c[3] for c in CASES])
def test_work_groups_hand_cases(v, shape, want, why):
    assert v.work_groups(*shape) == want, why


def test_work_groups_without_workspace_never_split():
    # A device with no K-split workspace runs every variant unsplit.
    v = fp32(32, 32, 32, sg=4)
    assert v.work_groups(256, 256, 4096, have_ws=False) == 64


def test_workspace_size_is_the_runtime_constant():
    # The clamp above assumes the runtime's 128 MiB workspace; the runtime
    # source states the same size.
    import os
    src = open(os.path.join(os.path.dirname(space.__file__), "csrc", "runtime.hip")).read()
    assert "kWsBytes = size_t(128) << 20" in src
    assert space.WORKSPACE_BYTES == 128 * MiB
