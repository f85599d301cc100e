"""CPU model of the register-staged kernels' global loads without masks.

Tiles whose slabs lie inside K run the register-staged loop without
per-element masks; rows past M read row M - 1 and load vectors that run past
N the row's last V columns (N >= V).  The two-deep prefetch loop
still issues the loads of one slab past the tile's last (they are never
staged), so those must go to the safe base address.  This test restates the
loads' index arithmetic and the PD = 1 / PD = 2 call sequences of
csrc/sgemm_variant.hip and checks that every dereferenced element lies inside
A (M x lda) and B (K x ldb) for every register-staged kernel of the family
(both load widths of LDS mode 1 and the scalar-load kernel of load-to-LDS
variants), on the last interior tile and on the first and last K split.

Tiles whose last slab runs past K (K not a multiple of the slab depth) run
the unmasked loop over their full slabs only and the masked loop over the
last one; the second test checks the unmasked phase of those tiles the same
way, and the third the tiles at the M and N edges of ragged shapes.
"""
import numpy as np
import pytest

from paper_2507_15277_amd import space
from paper_2507_15277_amd.tune import kernel_hash

# Build hash of the kernel source whose load arithmetic the model below was
# last checked against, line by line.  A change to the kernel source fails
# the first test until the model has been re-read against it.
MODELLED_KERNEL = "5462ee79f990"


def test_model_follows_the_current_kernel_source():
    assert kernel_hash() == MODELLED_KERNEL, (
        "csrc/sgemm_variant.hip changed since this load model was checked against it: re-check gload's "
        "clamps and the PD = 1 / PD = 2 call sequences, then update MODELLED_KERNEL")


def _loads(v, M, N, K, lda, ldb, tm, tn, kt0, kt1, V=None):
    V = V or v.vw
    KWG, NT = v.kwg, v.threads
    tid = np.arange(NT)

    def gload(kt, out):
        if not kt < kt1:           # past the last slab: the safe base address
            return
        for rows, vec_row, n_items, ld, base_r, base_c, name in (
                (v.mwg, KWG // V, v.mwg * (KWG // V), lda, tm * v.mwg, kt * KWG, "A"),
                (KWG, v.nwg // V, KWG * (v.nwg // V), ldb, kt * KWG, tn * v.nwg, "B")):
            items = np.concatenate([tid + i * NT for i in range(-(-n_items // NT))])
            items = items[items < n_items]
            r = base_r + items // vec_row
            c = base_c + (items % vec_row) * V
            if name == "A":
                r = np.minimum(r, M - 1)            # rows past M read row M - 1
            else:
                c = np.where(c + V <= N, c, N - V)  # vectors past N: the row's last V
            assert np.all(r >= 0) and np.all(c >= 0)
            out[name] = max(out[name], int(np.max(r * ld + c + V - 1)))

    out = {"A": -1, "B": -1}
    if v.pd == 1:
        gload(kt0, out)
        for kt in range(kt0, kt1):
            if kt + 1 < kt1:
                gload(kt + 1, out)
    else:
        gload(kt0, out)
        gload(kt0 + 1, out)
        kt = kt0
        while kt + 2 < kt1:
            gload(kt + 2, out)
            gload(kt + 3, out)
            kt += 2
    return out


def _staged_kernels():
    """(variant, vector width) of every kernel that stages through registers:
    both kernels of LDS mode 1, and the scalar-load kernel of LDS mode 2."""
    out = []
    for v in space.full_family():
        if v.prec == 0 and v.lds == 1:
            out += [(v, v.vw)] + ([(v, 1)] if v.vw != 1 else [])
        elif v.prec == 0 and v.lds == 2:
            out.append((v, 1))
    return out


def _split_ranges(v, M, N, nkt):
    """[kt0, kt1) of the first and last K split (the runtime's split count)."""
    splits = 1
    if v.sg > 1:
        sp = min(v.sg, nkt, space.WORKSPACE_BYTES // (M * N * 4))
        if sp >= 2:
            splits = -(-nkt // -(-nkt // sp))
    per = -(-nkt // splits)
    return {(part * per, min(nkt, part * per + per)) for part in {0, splits - 1}}


@pytest.mark.parametrize("shape", [(256, 256, 256), (512, 1024, 768)])
def test_interior_loads_stay_inside(shape):
    M, N, K = shape
    staged = _staged_kernels()
    assert any(vw == 1 for _, vw in staged) and any(v.lds == 2 for v, _ in staged)
    checked = 0
    for v, vw in staged:
        nbm, nbn = M // v.mwg, N // v.nwg
        if K % v.kwg or nbm == 0 or nbn == 0:
            continue
        for kt0, kt1 in _split_ranges(v, M, N, K // v.kwg):
            out = _loads(v, M, N, K, K, N, nbm - 1, nbn - 1, kt0, kt1, vw)
            assert out["A"] <= (M - 1) * K + K - 1, (v.name, vw, shape, kt0)
            assert out["B"] <= (K - 1) * N + N - 1, (v.name, vw, shape, kt0)
            checked += 1
    assert checked > 100


@pytest.mark.parametrize("shape", [(256, 256, 261), (512, 1024, 771), (257, 131, 1029)])
def test_k_tail_unmasked_phase_stays_inside(shape):
    M, N, K = shape
    checked = 0
    for v, vw in _staged_kernels():
        nbm, nbn = M // v.mwg, N // v.nwg
        nkt = -(-K // v.kwg)
        if K % v.kwg == 0 or nbm == 0 or nbn == 0:
            continue
        for kt0, kt1 in _split_ranges(v, M, N, nkt):
            if kt1 * v.kwg <= K or kt1 - 1 <= kt0:
                continue            # no tail slab, or the masked loop alone
            assert (kt1 - 1) * v.kwg <= K
            out = _loads(v, M, N, K, K, N, nbm - 1, nbn - 1, kt0, kt1 - 1, vw)
            assert out["A"] <= (M - 1) * K + K - 1, (v.name, vw, shape, kt0)
            assert out["B"] <= (K - 1) * N + N - 1, (v.name, vw, shape, kt0)
            checked += 1
    assert checked > 100


@pytest.mark.parametrize("shape", [(257, 131, 1029), (100, 1000, 300), (1000, 36, 64), (33, 4097, 515)])
def test_edge_tiles_stay_inside(shape):
    M, N, K = shape
    checked = 0
    for v, vw in _staged_kernels():
        nbm, nbn = -(-M // v.mwg), -(-N // v.nwg)
        nkt = -(-K // v.kwg)
        for tm, tn in {(nbm - 1, nbn - 1), (nbm - 1, 0), (0, nbn - 1)}:
            if N < vw:
                continue            # the masked loop
            for kt0, kt1 in _split_ranges(v, M, N, nkt):
                if kt1 * v.kwg > K:
                    kt1 -= 1        # the tail slab runs the masked loop
                if kt1 <= kt0:
                    continue
                out = _loads(v, M, N, K, K, N, tm, tn, kt0, kt1, vw)
                assert out["A"] <= (M - 1) * K + K - 1, (v.name, vw, shape, tm, tn, kt0)
                assert out["B"] <= (K - 1) * N + N - 1, (v.name, vw, shape, tm, tn, kt0)
                checked += 1
    assert checked > 100


def _vshift(v, s):
    """The kernel's vshift: element j takes element j + s; the last s keep v[-1]."""
    V = len(v)
    return [v[min(j + s, V - 1)] if j < V - 1 else v[V - 1] for j in range(V)]


@pytest.mark.parametrize("V", [2, 4])
@pytest.mark.parametrize("N", [4, 5, 6, 7, 33, 130, 131])
def test_straddling_vector_staged_in_place(V, N):
    # One row of B: every load vector of every tile column, with the address
    # rule of the loop without masks and the shift applied when staged, puts
    # B[n + j] at staged position j for every column n + j < N.
    if N < V:
        return
    row = np.arange(1000, 1000 + N)
    for NWG in (16, 64):
        for n0 in range(0, N, NWG):
            nshift = n0 + NWG > N and N % V != 0
            for nn in range(0, NWG, V):
                n = n0 + nn
                nr = n if n + V <= N else N - V
                assert 0 <= nr and nr + V <= N
                x = list(row[nr:nr + V])
                if nshift:
                    x = _vshift(x, n - (N - V) if n < N < n + V else 0)
                for j in range(V):
                    if n + j < N:
                        assert x[j] == row[n + j], (V, N, NWG, n0, nn, j)
