"""Variant space of the SGEMM kernel and the family that is compiled.

Sec. III-A: tuning parameters are compile-time constants and each parameter
combination compiled is a code variant.  Sec. V-C: the parameter space is too
large to explore fully, so the paper times the library's hand-tuned defaults
plus a random selection from the space.  This module does the same for the
gfx950 kernel in ``csrc/sgemm_variant.hip``: it enumerates every legal
configuration of the axes below, then keeps a fixed default, a hand-picked
set and a seeded sample stratified by work-group tile shape.

Axes (names match the kernel's FF_* macros):
  MWG, NWG  work-group tile; KWG slab depth; MI MFMA block edge (32: 32x32x2,
  16: 16x16x4); WM x WN wave grid; SK intra-work-group split of K; VW
  global-load vector width; LDS staging on/off; GM tile-order group height;
  SG largest number of work-groups splitting one tile's K range.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, asdict

import numpy as np

# Per-lane register budgets used to reject configurations that would spill
# or leave no room for the pipeline (gfx950: 512 VGPR+AGPR per lane at one
# wave per SIMD).
WORKSPACE_BYTES = 128 << 20  # per-device K-split workspace of the runtime
MAX_ACC = 128            # accumulator floats per lane
MAX_DIRECT_OPERANDS = 64  # double-buffered operand registers, direct loads
MAX_LDS_BYTES = 80 * 1024  # keeps >= 2 work-groups per CU possible (160 KB LDS)
MAX_DMA_LDS_BYTES = 160 * 1024  # load-to-LDS staging may fill the CU's LDS
MAX_THREADS = 512
MAX_STAGING = 64          # floats per thread held in flight between global loads and LDS


@dataclass(frozen=True)
class Variant:
    mwg: int
    nwg: int
    kwg: int
    mi: int
    wm: int
    wn: int
    sk: int
    vw: int
    lds: int
    gm: int = 8
    sg: int = 1
    prec: int = 0   # 0 FP32 MFMA; 1 bf16x3, 2 bf16x6, 3 scaled fp16, 4 scaled fp16 in two pieces (csrc/sgemm_split.hip)
    pd: int = 1     # prefetch depth in slabs (LDS-staged FP32 variants)

    @property
    def mk(self):
        if self.prec:
            return 16 if self.mi == 32 else 32
        return 2 if self.mi == 32 else 4

    @property
    def terms(self):
        return {0: 1, 1: 2, 2: 3, 3: 1, 4: 2}[self.prec]

    @property
    def source(self):
        return "sgemm_split.hip" if self.prec else "sgemm_variant.hip"

    @property
    def threads(self):
        return 64 * self.wm * self.wn * self.sk

    @property
    def rm(self):
        return self.mwg // (self.wm * self.mi)

    @property
    def rn(self):
        return self.nwg // (self.wn * self.mi)

    @property
    def steps(self):
        """MFMA steps per split group per slab."""
        return self.kwg // (self.sk * self.mk)

    @property
    def acc_regs(self):
        return self.rm * self.rn * self.mi * self.mi // 64

    @property
    def lds_bytes(self):
        if self.prec:
            stage = 2 * self.terms * (self.mwg + self.nwg) * (self.kwg + 8)     # bytes
            if self.lds == 2:
                return (self.pd + 1) * (-(-stage // 1024) * 1024) + 1024
            return 2 * stage
        stage = self.mwg * (self.kwg + 4) + self.kwg * (self.nwg + 4)
        red = (self.sk - 1) * self.mwg * self.nwg
        if self.lds == 2:
            # PD + 1 stages, each rounded up to whole 1 KB wave copies, plus
            # 1 KB for the surplus copies.
            stage_dma = -(-stage // 256) * 256
            return 4 * max((self.pd + 1) * stage_dma + 256, red)
        return 4 * (max(2 * stage, red) if self.lds else max(red, 1))

    @property
    def dma_copies(self):
        """Load-to-LDS copies per wave per slab (LDS mode 2)."""
        stage = self.mwg * (self.kwg + 4) + self.kwg * (self.nwg + 4)
        waves = self.wm * self.wn * self.sk
        return -(-(-(-stage // 256)) // waves)

    @property
    def name(self):
        if self.prec:
            form = PREC_NAMES[self.prec]
            n = f"sgemmx_{form}_m{self.mwg}n{self.nwg}k{self.kwg}_i{self.mi}_w{self.wm}x{self.wn}"
            return (n + (f"_p{self.sg}" if self.sg != 1 else "") + ("_l2" if self.lds == 2 else "")
                    + (f"_d{self.pd}" if self.pd != 1 else ""))
        n = (f"sgemm_m{self.mwg}n{self.nwg}k{self.kwg}_i{self.mi}_w{self.wm}x{self.wn}"
             f"_s{self.sk}_v{self.vw}_l{self.lds}")
        if self.gm != 8:
            n += f"_g{self.gm}"
        if self.sg != 1:
            n += f"_p{self.sg}"
        if self.pd != 1:
            n += f"_d{self.pd}"
        return n

    def defines(self):
        if self.prec:
            return {"FF_MWG": self.mwg, "FF_NWG": self.nwg, "FF_KWG": self.kwg, "FF_MI": self.mi,
                    "FF_WM": self.wm, "FF_WN": self.wn, "FF_PREC": self.prec, "FF_GM": self.gm,
                    "FF_SG": self.sg, "FF_LDS": self.lds, "FF_PD": self.pd, "FF_NAME": self.name}
        return {"FF_MWG": self.mwg, "FF_NWG": self.nwg, "FF_KWG": self.kwg, "FF_MI": self.mi,
                "FF_WM": self.wm, "FF_WN": self.wn, "FF_SK": self.sk, "FF_VW": self.vw,
                "FF_LDS": self.lds, "FF_GM": self.gm, "FF_SG": self.sg, "FF_PD": self.pd,
                "FF_NAME": self.name}

    def work_groups(self, M, N, K, have_ws=True):
        """Work-groups of this variant's GEMM launch on (M, N, K): tiles times
        K splits, the split count chosen as the runtime chooses it (as many
        as SG allows, no more than there are slabs, every split non-empty,
        within the 128 MiB workspace); 0 for an empty product."""
        if M <= 0 or N <= 0:
            return 0
        if self.prec and self.lds == 2:
            K = -(-K // 64) * 64          # pre-split forms run over K padded to 64
        nb = -(-M // self.mwg) * -(-N // self.nwg)
        nkt = -(-K // self.kwg)
        if self.sg > 1 and nkt > 1 and have_ws:
            sp = min(self.sg, nkt, WORKSPACE_BYTES // (M * N * 4))
            if sp >= 2 and nb * sp <= 2**31 - 1:
                per = -(-nkt // sp)
                return nb * -(-nkt // per)
        return nb

    def descriptor(self, vid):
        """Manifest / set-file descriptor: id name MWG NWG KWG MI WM WN SK VW LDS GM SG PREC PD."""
        return (f"{vid} {self.name} {self.mwg} {self.nwg} {self.kwg} {self.mi} {self.wm} {self.wn} "
                f"{self.sk} {self.vw} {self.lds} {self.gm} {self.sg} {self.prec} {self.pd}")

    def as_dict(self):
        return asdict(self)


PREC_NAMES = {0: "fp32", 1: "bf16x3", 2: "bf16x6", 3: "fp16s", 4: "fp16x3"}
MAX_SPLIT_LDS_BYTES = 160 * 1024


def legal_split(v: Variant) -> bool:
    """Constraints of the split-precision kernel (csrc/sgemm_split.hip)."""
    if v.mi not in (16, 32) or v.sk != 1 or v.sg not in SPLITS or v.lds not in (1, 2) or v.vw != 4:
        return False
    if v.pd not in (1, 2) or (v.pd == 2 and v.lds != 2):
        return False
    if v.mwg % (v.wm * v.mi) or v.nwg % (v.wn * v.mi) or v.kwg % v.mk:
        return False
    if v.threads > MAX_THREADS or v.acc_regs > MAX_ACC or v.lds_bytes > MAX_SPLIT_LDS_BYTES:
        return False
    if v.lds == 2:
        # Pre-split: K is padded to 64, so a slab must divide it.
        return 64 % v.kwg == 0
    # Staged FP32 slab values per thread (8 per load item).
    if (v.mwg + v.nwg) * v.kwg > MAX_STAGING * v.threads:
        return False
    return True


def legal(v: Variant) -> bool:
    """Constraints of the kernel template plus resource budgets."""
    if v.prec:
        return legal_split(v)
    if v.mi not in (16, 32) or v.vw not in (1, 2, 4) or v.lds not in (0, 1, 2):
        return False
    if v.sg not in SPLITS or v.pd not in (1, 2) or (v.pd == 2 and not v.lds):
        return False
    if v.lds == 2 and (v.vw != 4 or (v.pd - 1) * v.dma_copies > 63):
        return False
    if v.mwg % (v.wm * v.mi) or v.nwg % (v.wn * v.mi):
        return False
    if v.kwg % (v.sk * v.mk) or v.kwg % 4 or v.nwg % 4:
        return False
    lds_cap = MAX_DMA_LDS_BYTES if v.lds == 2 else MAX_LDS_BYTES
    if v.threads > MAX_THREADS or v.acc_regs > MAX_ACC or v.lds_bytes > lds_cap:
        return False
    if max(v.mwg, v.nwg) > 4 * min(v.mwg, v.nwg):
        return False  # elongated tiles re-read the long operand too often
    if not v.lds and 2 * v.steps * (v.rm + v.rn) > MAX_DIRECT_OPERANDS:
        return False
    if v.lds:
        # Every thread should have at least one vector of each slab to stage,
        # and the staged slab must fit in registers next to the accumulators.
        if v.mwg * v.kwg < v.threads * v.vw or v.kwg * v.nwg < v.threads * v.vw:
            return False
        if v.pd * (v.mwg * v.kwg + v.kwg * v.nwg) > MAX_STAGING * v.threads:
            return False
    return True


TILES = (16, 32, 64, 128, 256)
KSTEPS = (8, 16, 32, 64, 128)
SPLITS = (1, 2, 4, 8, 16)


def enumerate_space():
    """All legal configurations, in a fixed order."""
    out = []
    for mi, mwg, nwg, kwg, wm, wn, sk, vw, lds, sg, pd in itertools.product(
            (32, 16), TILES, TILES, KSTEPS, (1, 2, 4), (1, 2, 4), (1, 2, 4), (1, 2, 4), (1, 0, 2),
            SPLITS, (1, 2)):
        v = Variant(mwg, nwg, kwg, mi, wm, wn, sk, vw, lds, 8, sg, 0, pd)
        if legal(v):
            out.append(v)
    return out


# The fixed single variant of the first workload: 64x64 tile, K-step 16.
DEFAULT = Variant(64, 64, 16, 32, 2, 2, 1, 4, 1)

# Hand-picked configurations that cover large, skinny and tiny shapes.
HAND = [
    Variant(128, 128, 16, 32, 2, 2, 1, 4, 1),
    Variant(128, 128, 32, 32, 2, 2, 1, 4, 1),
    Variant(128, 128, 16, 32, 2, 2, 2, 4, 1),
    Variant(256, 128, 16, 32, 4, 2, 1, 4, 1),
    Variant(128, 256, 16, 32, 2, 4, 1, 4, 1),
    Variant(256, 128, 16, 32, 2, 2, 1, 4, 1),
    Variant(128, 256, 16, 32, 2, 2, 1, 4, 1),
    Variant(256, 256, 8, 32, 2, 4, 1, 4, 1),
    Variant(128, 64, 16, 32, 2, 2, 1, 4, 1),
    Variant(64, 128, 16, 32, 2, 2, 1, 4, 1),
    Variant(64, 64, 32, 32, 2, 2, 2, 4, 1),
    Variant(64, 64, 32, 32, 1, 1, 4, 4, 1),
    Variant(64, 64, 16, 16, 2, 2, 1, 4, 1),
    Variant(32, 32, 32, 32, 1, 1, 4, 4, 1),
    Variant(32, 32, 16, 16, 2, 2, 1, 1, 1),
    Variant(32, 32, 32, 16, 1, 1, 4, 4, 0),
    Variant(32, 64, 16, 32, 1, 2, 2, 2, 1),
    Variant(64, 32, 16, 32, 2, 1, 2, 2, 1),
    Variant(16, 16, 32, 16, 1, 1, 4, 4, 0),
    Variant(32, 32, 16, 32, 1, 1, 1, 4, 0),
    Variant(64, 64, 16, 32, 2, 2, 1, 4, 0),
    Variant(128, 128, 16, 16, 2, 2, 1, 4, 1),
    # K split over work-groups, for shapes with few tiles and long K.
    Variant(64, 64, 32, 32, 2, 2, 2, 4, 1, sg=2),
    Variant(64, 64, 32, 32, 2, 2, 2, 4, 1, sg=4),
    Variant(64, 64, 32, 32, 2, 2, 2, 4, 1, sg=8),
    Variant(64, 64, 16, 32, 2, 2, 1, 4, 1, sg=4),
    Variant(32, 32, 32, 32, 1, 1, 4, 4, 1, sg=4),
    Variant(32, 32, 32, 32, 1, 1, 4, 4, 1, sg=8),
    Variant(32, 32, 32, 32, 1, 1, 4, 4, 1, sg=16),
    Variant(16, 16, 32, 16, 1, 1, 2, 4, 0, sg=4),
    Variant(16, 16, 32, 16, 1, 1, 2, 4, 0, sg=16),
    Variant(128, 128, 16, 32, 2, 2, 1, 4, 1, sg=2),
    Variant(128, 128, 16, 32, 2, 2, 1, 4, 1, sg=4),
    Variant(256, 128, 16, 32, 4, 2, 1, 4, 1, sg=2),
    Variant(128, 64, 16, 32, 2, 2, 1, 4, 1, sg=4),
    Variant(64, 32, 32, 16, 2, 1, 2, 4, 1, sg=4),
    Variant(64, 32, 32, 16, 2, 1, 2, 4, 1, sg=8),
    # Deep K steps for small tiles: fewer global-load round trips.
    Variant(16, 16, 64, 16, 1, 1, 4, 4, 0),
    Variant(16, 16, 128, 16, 1, 1, 4, 4, 0),
    Variant(16, 32, 64, 16, 1, 1, 4, 2, 0),
    Variant(16, 32, 128, 16, 1, 1, 4, 4, 0),
    Variant(32, 32, 64, 16, 1, 1, 4, 4, 0),
    Variant(32, 32, 128, 32, 1, 1, 4, 4, 0),
    Variant(32, 32, 64, 32, 1, 1, 4, 4, 1),
    Variant(16, 16, 128, 16, 1, 1, 4, 4, 0, sg=4),
    Variant(32, 32, 128, 32, 1, 1, 4, 4, 0, sg=4),
    # Prefetch depth 2 (and deeper slabs) for the LDS-staged shapes that win
    # most often.
    Variant(32, 32, 64, 32, 1, 1, 4, 4, 1, pd=2),
    Variant(32, 32, 128, 32, 1, 1, 4, 4, 1),
    Variant(32, 32, 32, 32, 1, 1, 4, 4, 1, pd=2),
    Variant(64, 64, 32, 32, 2, 2, 2, 4, 1, pd=2),
    Variant(64, 64, 64, 32, 2, 2, 2, 4, 1),
    Variant(64, 64, 64, 32, 2, 2, 2, 4, 1, pd=2),
    Variant(64, 64, 64, 32, 2, 2, 1, 4, 1, pd=2),
    Variant(64, 64, 16, 32, 2, 2, 1, 4, 1, sg=4, pd=2),
    Variant(64, 64, 32, 32, 2, 2, 2, 4, 1, sg=8, pd=2),
    Variant(128, 128, 32, 32, 2, 2, 2, 4, 1, pd=2),
    Variant(128, 128, 32, 32, 2, 2, 1, 4, 1, pd=2),
    Variant(128, 128, 16, 32, 2, 2, 2, 4, 1, pd=2),
    Variant(256, 128, 16, 32, 4, 2, 1, 4, 1, pd=2),
    Variant(128, 256, 16, 32, 2, 4, 1, 4, 1, pd=2),
    Variant(64, 128, 32, 16, 4, 2, 1, 4, 1, sg=4, pd=2),
    Variant(64, 128, 32, 32, 1, 4, 1, 4, 1, sg=4, pd=2),
    Variant(256, 128, 16, 32, 4, 2, 1, 4, 1, sg=2, pd=2),
    # Load-to-LDS staging (LDS mode 2) for the frequent winners.
    Variant(64, 64, 64, 32, 2, 2, 2, 4, 2),
    Variant(64, 64, 64, 32, 2, 2, 2, 4, 2, pd=2),
    Variant(64, 64, 32, 32, 2, 2, 2, 4, 2),
    Variant(64, 64, 32, 32, 2, 2, 2, 4, 2, pd=2),
    Variant(64, 64, 128, 32, 2, 2, 2, 4, 2),
    Variant(32, 32, 128, 32, 1, 1, 4, 4, 2),
    Variant(32, 32, 128, 32, 1, 1, 4, 4, 2, pd=2),
    Variant(128, 128, 32, 32, 2, 2, 2, 4, 2),
    Variant(128, 128, 32, 32, 2, 2, 2, 4, 2, pd=2),
    Variant(128, 128, 64, 32, 2, 2, 2, 4, 2),
    Variant(256, 128, 16, 32, 4, 2, 1, 4, 2),
    Variant(256, 128, 16, 32, 4, 2, 1, 4, 2, pd=2),
    Variant(256, 128, 32, 32, 4, 2, 1, 4, 2),
    Variant(128, 256, 16, 32, 2, 4, 1, 4, 2, pd=2),
    Variant(64, 64, 32, 32, 2, 2, 2, 4, 2, sg=8, pd=2),
    Variant(16, 32, 128, 16, 1, 1, 4, 4, 2, sg=4),
    Variant(64, 128, 32, 32, 1, 4, 1, 4, 2, pd=2),
    # Larger tiles and deeper slabs with load-to-LDS staging.
    Variant(256, 256, 32, 16, 2, 4, 1, 4, 2),
    Variant(256, 256, 16, 16, 2, 4, 1, 4, 2, pd=2),
    Variant(256, 256, 32, 32, 4, 2, 1, 4, 2),
    Variant(256, 128, 32, 32, 4, 2, 1, 4, 2, pd=2),
    Variant(128, 256, 32, 32, 2, 4, 1, 4, 2),
    Variant(128, 128, 64, 32, 2, 2, 1, 4, 2),
    Variant(64, 64, 128, 32, 2, 2, 2, 4, 2, sg=4),
    Variant(64, 64, 64, 32, 2, 2, 2, 4, 2, sg=8),
    Variant(64, 128, 64, 32, 2, 2, 2, 4, 2),
    Variant(128, 64, 64, 32, 2, 2, 2, 4, 2),
    Variant(32, 32, 128, 32, 1, 1, 4, 4, 2, sg=4),
    Variant(32, 16, 128, 16, 1, 1, 4, 4, 2),
]


def family(n=320, seed=0):
    """The compiled family: DEFAULT, HAND, then a seeded sample stratified by
    (MWG, NWG) tile shape, up to ``n`` variants.  Deterministic for a seed."""
    space = enumerate_space()
    legal_set = set(space)
    chosen = [DEFAULT] + [v for v in HAND if v in legal_set and v != DEFAULT]
    seen = set(chosen)
    strata = {}
    for v in space:
        if v not in seen:
            strata.setdefault((v.mwg, v.nwg), []).append(v)
    rng = np.random.default_rng([11, seed])
    keys = sorted(strata)
    for k in keys:
        order = rng.permutation(len(strata[k]))
        strata[k] = [strata[k][i] for i in order]
    # Round-robin over strata so every tile shape is represented.
    idx = 0
    while len(chosen) < n and any(strata[k] for k in keys):
        k = keys[idx % len(keys)]
        if strata[k]:
            v = strata[k].pop()
            chosen.append(v)
            seen.add(v)
        idx += 1
    return chosen[:n]


# Split-precision family: the same handful of work-group shapes for each form.
SPLIT_SHAPES = [
    # (MWG, NWG, KWG, MI, WM, WN)
    (128, 128, 32, 32, 2, 2),
    (128, 128, 16, 32, 2, 2),
    (256, 128, 16, 32, 4, 2),
    (128, 256, 16, 32, 2, 4),
    (64, 64, 32, 32, 2, 2),
    (64, 64, 64, 32, 2, 2),
    (64, 128, 32, 32, 2, 2),
    (128, 64, 32, 32, 2, 2),
    (32, 32, 64, 32, 1, 1),
    (32, 32, 32, 16, 2, 2),
    (64, 64, 32, 16, 2, 2),
    (128, 128, 32, 16, 4, 4),
]


# Split-precision shapes with the K range split over work-groups, for the
# shapes with few tiles and long K.  (MWG, NWG, KWG, MI, WM, WN, SG)
SPLIT_K_SHAPES = [
    (64, 64, 32, 32, 2, 2, 4),
    (64, 64, 64, 32, 2, 2, 8),
    (128, 128, 32, 32, 2, 2, 4),
    (32, 32, 64, 32, 1, 1, 8),
    (32, 32, 32, 16, 2, 2, 4),
    (64, 64, 32, 16, 2, 2, 8),
]


# Pre-split shapes (LDS mode 2: pieces formed once per call, copied to LDS).
PRESPLIT_SHAPES = [
    # (MWG, NWG, KWG, MI, WM, WN, SG, PD)
    (128, 128, 32, 32, 2, 2, 1, 1),
    (128, 128, 64, 32, 2, 2, 1, 1),
    (256, 128, 32, 32, 4, 2, 1, 1),
    (128, 256, 32, 32, 2, 4, 1, 1),
    (256, 256, 32, 32, 4, 2, 1, 1),
    (64, 64, 64, 32, 2, 2, 1, 1),
    (64, 64, 64, 32, 2, 2, 8, 1),
    (128, 128, 32, 32, 2, 2, 4, 1),
    (128, 128, 64, 16, 4, 4, 1, 1),
    (32, 32, 64, 32, 1, 1, 8, 1),
    (128, 128, 32, 32, 2, 2, 1, 2),
    (128, 128, 64, 32, 2, 2, 1, 2),
    (256, 128, 32, 32, 4, 2, 1, 2),
    (128, 256, 32, 32, 2, 4, 1, 2),
    (256, 256, 32, 32, 4, 2, 1, 2),
    (64, 64, 64, 32, 2, 2, 8, 2),
    (128, 128, 32, 32, 2, 2, 4, 2),
    (128, 128, 16, 32, 2, 2, 1, 2),
    # Eight waves (two per SIMD) and K-step 16, for the three-piece form's LDS budget.
    (128, 128, 32, 32, 4, 2, 1, 1),
    (128, 128, 32, 32, 4, 2, 1, 2),
    (128, 128, 16, 32, 4, 2, 1, 2),
    (256, 128, 16, 32, 4, 2, 1, 1),
    (256, 128, 16, 32, 4, 2, 1, 2),
    (128, 256, 16, 32, 2, 4, 1, 1),
    (64, 64, 64, 32, 2, 2, 4, 2),
    # Larger blocks per wave (128 x 64 or 64 x 128: fewer fragment reads per MFMA).
    (256, 128, 16, 32, 2, 2, 1, 1),
    (256, 128, 32, 32, 2, 2, 1, 1),
    (128, 256, 16, 32, 2, 2, 1, 1),
    (256, 128, 16, 32, 2, 2, 1, 2),
]


def split_family(precs=(1, 2, 3)):
    out = []
    for prec in precs:
        for (mwg, nwg, kwg, mi, wm, wn) in SPLIT_SHAPES:
            v = Variant(mwg, nwg, kwg, mi, wm, wn, 1, 4, 1, 8, 1, prec)
            if legal(v):
                out.append(v)
    # Later lists follow, shape by shape with the forms inside, so a shape
    # appended to a list adds ids at the end and earlier ids keep their
    # variants (tables and set files refer to variants by id).
    for (mwg, nwg, kwg, mi, wm, wn, sg) in SPLIT_K_SHAPES:
        for prec in precs:
            v = Variant(mwg, nwg, kwg, mi, wm, wn, 1, 4, 1, 8, sg, prec)
            if legal(v):
                out.append(v)
    for (mwg, nwg, kwg, mi, wm, wn, sg, pd) in PRESPLIT_SHAPES:
        for prec in precs:
            v = Variant(mwg, nwg, kwg, mi, wm, wn, 1, 4, 2, 8, sg, prec, pd)
            if legal(v):
                out.append(v)
    return out


# FP32 variants added after the split forms (ids after theirs, so earlier
# ids keep their variants): eight-wave K splits of 16- and 32-wide tiles
# (SK 8, outside the sampled space's SK range), for small M and N with long K;
# then 16x16-block versions of the winning tile shapes, where each wave holds
# several independent accumulator blocks instead of one 32x32 chain whose
# back-to-back MFMAs wait on each other.
EXTRA_FP32 = [
    Variant(16, 16, 128, 16, 1, 1, 8, 4, 0),
    Variant(16, 16, 256, 16, 1, 1, 8, 4, 0),
    Variant(16, 16, 128, 16, 1, 1, 8, 4, 2),
    Variant(16, 16, 256, 16, 1, 1, 8, 4, 2),
    Variant(16, 32, 128, 16, 1, 1, 8, 4, 2),
    Variant(32, 16, 128, 16, 1, 1, 8, 4, 2),
    Variant(16, 16, 128, 16, 1, 1, 8, 4, 1, pd=2),
    Variant(16, 16, 256, 16, 1, 1, 8, 4, 1),
    Variant(32, 32, 128, 16, 1, 1, 8, 4, 2),
    Variant(32, 32, 128, 32, 1, 1, 8, 4, 2),
    Variant(32, 32, 256, 32, 1, 1, 8, 4, 2),
    Variant(64, 64, 64, 16, 2, 2, 2, 4, 1, pd=2),
    Variant(64, 64, 64, 16, 2, 2, 2, 4, 1),
    Variant(64, 64, 32, 16, 2, 2, 1, 4, 1, pd=2),
    Variant(64, 64, 32, 16, 2, 2, 2, 4, 1, pd=2),
    Variant(64, 64, 64, 16, 2, 2, 1, 4, 1, pd=2),
    Variant(64, 64, 16, 16, 2, 2, 1, 4, 1, pd=2),
    Variant(32, 32, 64, 16, 1, 1, 4, 4, 1, pd=2),
    Variant(32, 32, 32, 16, 1, 1, 4, 4, 1, pd=2),
    Variant(32, 32, 64, 16, 1, 1, 2, 4, 1, pd=2),
    Variant(64, 128, 32, 16, 2, 2, 2, 4, 1, pd=2),
    Variant(128, 64, 32, 16, 2, 2, 2, 4, 1, pd=2),
    Variant(128, 128, 32, 16, 2, 2, 2, 4, 1, pd=2),
    Variant(128, 128, 32, 16, 2, 2, 1, 4, 1, pd=2),
    Variant(128, 128, 32, 16, 2, 2, 1, 4, 2, pd=2),
    Variant(128, 256, 16, 16, 2, 4, 1, 4, 1, pd=2),
    Variant(128, 256, 16, 16, 2, 4, 1, 4, 1),
    Variant(256, 256, 32, 16, 4, 2, 1, 4, 2),
]


def full_family():
    """Everything that is compiled: the FP32 family, then the split forms
    (appended, so FP32 variant ids do not depend on the split family), then
    the two-piece scaled FP16 form and the later FP32 additions, each added
    last so that earlier ids keep their variants."""
    return family() + split_family() + split_family(precs=(4,)) + [v for v in EXTRA_FP32 if legal(v)]
