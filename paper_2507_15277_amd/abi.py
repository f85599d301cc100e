"""Thin ctypes binding of libfewfit.so (C ABI in include/fewfit.h).

Argument marshalling only: every function forwards to the native entry point
of the same name.  Matrices may be given as torch tensors (their device
address is passed) or as raw integer addresses; ``stream`` defaults to
torch's current HIP stream.  A negative status raises :class:`FewfitError`
carrying the library's error text.  If the library has not been built the
first call raises: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfewfit.so")

_lib = None

FF_OK = 0
FF_ERR_M, FF_ERR_N, FF_ERR_K = -1, -2, -3
FF_ERR_A, FF_ERR_LDA, FF_ERR_B, FF_ERR_LDB, FF_ERR_C, FF_ERR_LDC = -5, -6, -7, -8, -10, -11
FF_ERR_NO_SET, FF_ERR_VARIANT, FF_ERR_PARSE = -100, -101, -102
FF_ERR_ARCH, FF_ERR_HIP, FF_ERR_IO, FF_ERR_TOO_LARGE, FF_ERR_ARG = -103, -104, -105, -106, -107
FF_FORM_FP32, FF_FORM_BF16X3, FF_FORM_BF16X6, FF_FORM_FP16S, FF_FORM_FP16X3 = 0, 1, 2, 3, 4
FORM_NAMES = ("fp32", "bf16x3", "bf16x6", "fp16s", "fp16x3")   # a variant's precision form
FF_FORM_MIXED = 5            # the set slot whose members may be of any form
SET_FORMS = FORM_NAMES + ("mixed",)

EXPORTS = ("sgemm", "sgemm_form", "variant_set_load", "variant_select", "variant_select_form",
           "fewfit_last_error",
           "variant_manifest_load", "variant_count", "variant_info", "sgemm_variant",
           "sgemm_time", "screen_reference", "screen_compare", "ptune_postprocess",
           "ptune_cost", "ptune_select", "ptune_assign", "ptune_nearest", "ptune_dispatch",
           "ptune_select_total", "ptune_kmeans", "ptune_tree", "ptune_tree_route", "sgemm_grouped_plan",
           "sgemm_grouped", "variant_work_groups", "sgemm_form_noalloc")


class FewfitError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fewfit error {code}: {msg}")
        self.code = code


def lib():
    """Load libfewfit.so (torch first, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2507_15277_amd.build` "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        i64, f32, f64, vp, i32 = ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        gemm_args = [i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, vp]
        L.sgemm.argtypes = gemm_args
        L.sgemm_form.argtypes = [i32] + gemm_args
        L.sgemm_form_noalloc.argtypes = [i32] + gemm_args
        L.variant_select_form.argtypes = [i32, i64, i64, i64]
        L.sgemm_variant.argtypes = [i32] + gemm_args
        L.sgemm_time.argtypes = [i32] + gemm_args + [i32, i32, i32, vp]
        L.variant_work_groups.argtypes = [i32, i64, i64, i64, vp]
        L.variant_set_load.argtypes = [ctypes.c_char_p]
        L.variant_manifest_load.argtypes = [ctypes.c_char_p]
        L.variant_select.argtypes = [i64, i64, i64]
        L.variant_count.argtypes = []
        L.variant_info.argtypes = [i32, ctypes.c_char_p, ctypes.c_size_t]
        L.fewfit_last_error.argtypes = []
        L.fewfit_last_error.restype = ctypes.c_char_p
        L.screen_reference.argtypes = [i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, vp, vp, vp]
        L.screen_compare.argtypes = [i64, i64, vp, i64, vp, vp, f64, vp, vp, vp, vp, vp]
        L.ptune_postprocess.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
        L.ptune_cost.argtypes = [i32, i32, vp, i32, vp, i32, vp, vp]
        L.ptune_select.argtypes = [i32, i32, vp, i32, vp, i32, i32, vp, vp, vp]
        L.ptune_assign.argtypes = [i32, i32, vp, i32, vp, i32, vp, vp]
        L.ptune_nearest.argtypes = [i32, vp, i64, i64, i64]
        L.ptune_dispatch.argtypes = [i32, vp, i32, vp, vp, vp, vp, i32, i64, i64, i64]
        L.sgemm_grouped_plan.argtypes = [i32, i32, vp, vp, vp]
        L.sgemm_grouped.argtypes = [i32, i32, vp, vp, i32, f32, f32, i32, vp]
        L.ptune_select_total.argtypes = [i32, i32, vp, i32, vp, vp, i32, i32, vp, vp, vp]
        L.ptune_kmeans.argtypes = [i32, i32, vp, i32, vp, i32, vp, i32, vp, vp, vp]
        L.ptune_tree.argtypes = [i32, i32, vp, i32, vp, i32, vp, i32, vp, vp, vp, vp, vp, vp]
        L.ptune_tree_route.argtypes = [i32, vp, vp, vp, i32, vp]
        for name in EXPORTS:
            if name != "fewfit_last_error":
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def last_error() -> str:
    return lib().fewfit_last_error().decode()


def _check(rc):
    if rc < 0:
        raise FewfitError(rc, last_error())
    return rc


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# --- hot path ------------------------------------------------------------------

def sgemm(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    return _check(lib().sgemm(M, N, K, alpha, _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C), ldc,
                              _stream(stream)))


def sgemm_form(form, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    return _check(lib().sgemm_form(form, M, N, K, alpha, _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C), ldc,
                                   _stream(stream)))


def sgemm_form_noalloc(form, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    return _check(lib().sgemm_form_noalloc(form, M, N, K, alpha, _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C), ldc,
                                           _stream(stream)))


def variant_select_form(form, M, N, K):
    return _check(lib().variant_select_form(form, M, N, K))


def variant_set_load(path):
    return _check(lib().variant_set_load(os.fsencode(path)))


def variant_select(M, N, K):
    return _check(lib().variant_select(M, N, K))


# --- tuning ABI ----------------------------------------------------------------

def variant_manifest_load(directory):
    return _check(lib().variant_manifest_load(os.fsencode(directory)))


def variant_count():
    return _check(lib().variant_count())


def variant_info(vid):
    buf = ctypes.create_string_buffer(512)
    _check(lib().variant_info(vid, buf, len(buf)))
    return buf.value.decode()


def sgemm_variant(vid, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    return _check(lib().sgemm_variant(vid, M, N, K, alpha, _ptr(A), lda, _ptr(B), ldb, beta,
                                      _ptr(C), ldc, _stream(stream)))


def variant_work_groups(vid, M, N, K):
    out = ctypes.c_int64(0)
    _check(lib().variant_work_groups(vid, M, N, K, ctypes.byref(out)))
    return out.value


def sgemm_time(vid, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None,
               warmup=3, reps=10, trials=5):
    out = (ctypes.c_float * trials)()
    _check(lib().sgemm_time(vid, M, N, K, alpha, _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C), ldc,
                            _stream(stream), warmup, reps, trials, out))
    return list(out)


def screen_reference(M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc0, ref, tol, stream=None):
    return _check(lib().screen_reference(M, N, K, alpha, _ptr(A), lda, _ptr(B), ldb, beta,
                                         _ptr(C0), ldc0, _ptr(ref), _ptr(tol), _stream(stream)))


def screen_compare(M, N, C, ldc, ref, tol, stream=None, tol_scale=1.0, norms=False):
    """(bad count, max error/bound ratio[, normwise relative error])."""
    nbad = ctypes.c_int64(0)
    ratio = ctypes.c_double(0.0)
    e2 = ctypes.c_double(0.0)
    r2 = ctypes.c_double(0.0)
    _check(lib().screen_compare(M, N, _ptr(C), ldc, _ptr(ref), _ptr(tol), float(tol_scale),
                                ctypes.byref(nbad), ctypes.byref(ratio), ctypes.byref(e2),
                                ctypes.byref(r2), _stream(stream)))
    if norms:
        rel = (e2.value / r2.value) ** 0.5 if r2.value > 0 else 0.0
        return nbad.value, ratio.value, rel
    return nbad.value, ratio.value


# --- grouped launches ------------------------------------------------------------

def gemm_desc_dtype():
    """numpy layout of ff_gemm_desc (64 bytes)."""
    import numpy as np
    return np.dtype([("A", np.uint64), ("B", np.uint64), ("C", np.uint64), ("lda", np.int64),
                     ("ldb", np.int64), ("ldc", np.int64), ("M", np.int32), ("N", np.int32),
                     ("K", np.int32), ("tiles", np.int32)])


def sgemm_grouped_plan(vid, descs):
    """descs: numpy array of gemm_desc_dtype (modified in place: tiles).
    Returns (total tiles, prefix int32 array, vector loads allowed)."""
    import numpy as np
    prefix = np.empty(len(descs), np.int32)
    vec = ctypes.c_int(0)
    total = _check(lib().sgemm_grouped_plan(vid, len(descs), descs.ctypes.data, prefix.ctypes.data,
                                            ctypes.byref(vec)))
    return total, prefix, bool(vec.value)


def sgemm_grouped(vid, count, descs_dev, prefix_dev, total, alpha, beta, vec, stream=None):
    return _check(lib().sgemm_grouped(vid, count, _ptr(descs_dev), _ptr(prefix_dev), total, alpha, beta,
                                      1 if vec else 0, _stream(stream)))


# --- portability tuning (host) -------------------------------------------------

def _table(t):
    import numpy as np
    t = np.ascontiguousarray(t, dtype=np.float64)
    if t.ndim != 2:
        raise ValueError("table must be 2-D (variants x shapes)")
    return t


def _shapes(shapes):
    import numpy as np
    if shapes is None:
        return None, 0
    s = np.ascontiguousarray(shapes, dtype=np.int32)
    return s, s.size


def ptune_postprocess(t):
    import numpy as np
    t = _table(t)
    nv, ns = t.shape
    best, worst = np.empty(ns), np.empty(ns)
    best_id = np.empty(ns, np.int32)
    slow, speed = np.empty((nv, ns)), np.empty((nv, ns))
    _check(lib().ptune_postprocess(nv, ns, t.ctypes.data, best.ctypes.data, worst.ctypes.data,
                                   best_id.ctypes.data, slow.ctypes.data, speed.ctypes.data))
    return best, worst, best_id, slow, speed


def ptune_cost(t, kappa, shapes=None):
    import numpy as np
    t = _table(t)
    nv, ns = t.shape
    k = np.ascontiguousarray(kappa, dtype=np.int32)
    s, nsel = _shapes(shapes)
    out = ctypes.c_double(0.0)
    _check(lib().ptune_cost(nv, ns, t.ctypes.data, k.size, k.ctypes.data, nsel,
                            None if s is None else s.ctypes.data, ctypes.byref(out)))
    return out.value


def ptune_select(t, k, shapes=None, method=-1):
    import numpy as np
    t = _table(t)
    nv, ns = t.shape
    s, nsel = _shapes(shapes)
    kap = np.empty(k, np.int32)
    cost = ctypes.c_double(0.0)
    evals = ctypes.c_int64(0)
    n = _check(lib().ptune_select(nv, ns, t.ctypes.data, nsel, None if s is None else s.ctypes.data,
                                  k, method, kap.ctypes.data, ctypes.byref(cost), ctypes.byref(evals)))
    return tuple(int(x) for x in kap[:n]), cost.value, evals.value


def ptune_assign(t, kappa, shapes=None):
    import numpy as np
    t = _table(t)
    nv, ns = t.shape
    k = np.ascontiguousarray(kappa, dtype=np.int32)
    s, nsel = _shapes(shapes)
    n_out = ns if s is None else nsel
    win = np.empty(n_out, np.int32)
    _check(lib().ptune_assign(nv, ns, t.ctypes.data, k.size, k.ctypes.data, nsel,
                              None if s is None else s.ctypes.data, win.ctypes.data))
    return [int(x) for x in win]


def ptune_nearest(train_shapes, M, N, K):
    import numpy as np
    tr = np.ascontiguousarray(train_shapes, dtype=np.int64).reshape(-1, 3)
    return _check(lib().ptune_nearest(tr.shape[0], tr.ctypes.data, M, N, K))


def ptune_dispatch(train_shapes, members, cost, M, N, K, groups_train=None, groups_query=None, cus=0):
    """cost: ntrain x k log-slowdowns of the members on the training shapes;
    groups_train (ntrain x k) and groups_query (k): work-groups of each
    member's launch, for the wave correction on ``cus`` compute units."""
    import numpy as np
    tr = np.ascontiguousarray(train_shapes, dtype=np.int64).reshape(-1, 3)
    mem = np.ascontiguousarray(members, dtype=np.int32)
    c = np.ascontiguousarray(cost, dtype=np.float64).reshape(tr.shape[0], mem.size)
    gt = gq = None
    if groups_train is not None and groups_query is not None:
        gt = np.ascontiguousarray(groups_train, dtype=np.int64).reshape(tr.shape[0], mem.size)
        gq = np.ascontiguousarray(groups_query, dtype=np.int64).reshape(mem.size)
    return _check(lib().ptune_dispatch(tr.shape[0], tr.ctypes.data, mem.size, mem.ctypes.data,
                                       c.ctypes.data, None if gt is None else gt.ctypes.data,
                                       None if gq is None else gq.ctypes.data, cus, M, N, K))


def ptune_select_total(t, k, shapes, weights, method=-1):
    import numpy as np
    t = _table(t)
    nv, ns = t.shape
    s, nsel = _shapes(shapes)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    kap = np.empty(k, np.int32)
    tot = ctypes.c_double(0.0)
    evals = ctypes.c_int64(0)
    n = _check(lib().ptune_select_total(nv, ns, t.ctypes.data, nsel, s.ctypes.data, w.ctypes.data, k, method,
                                        kap.ctypes.data, ctypes.byref(tot), ctypes.byref(evals)))
    return tuple(int(x) for x in kap[:n]), tot.value, evals.value


def ptune_kmeans(t, k, shapes, init, max_iter=100):
    import numpy as np
    t = _table(t)
    nv, ns = t.shape
    s, nsel = _shapes(shapes)
    ini = np.ascontiguousarray(init, dtype=np.int32)
    kap = np.empty(k, np.int32)
    n_pts = ns if s is None else nsel
    asg = np.empty(n_pts, np.int32)
    it = ctypes.c_int(0)
    n = _check(lib().ptune_kmeans(nv, ns, t.ctypes.data, nsel, None if s is None else s.ctypes.data, k,
                                  ini.ctypes.data, max_iter, kap.ctypes.data, asg.ctypes.data, ctypes.byref(it)))
    return tuple(int(x) for x in kap[:n]), [int(a) for a in asg], it.value


def ptune_tree(t, k, shapes, features, model=False):
    """(kappa, leaf of each shape); with model=True also the tree
    (node_feat, node_thr, node_child) and each leaf's variant."""
    import numpy as np
    t = _table(t)
    nv, ns = t.shape
    s, nsel = _shapes(shapes)
    f = np.ascontiguousarray(features, dtype=np.float64)
    kap = np.empty(k, np.int32)
    n_pts = ns if s is None else nsel
    leaf = np.empty(n_pts, np.int32)
    nf = np.full(2 * k - 1, -2, np.int32)
    nt = np.zeros(2 * k - 1, np.float64)
    nc = np.full(2 * (2 * k - 1), -2, np.int32)
    lv = np.full(k, -1, np.int32)
    n = _check(lib().ptune_tree(nv, ns, t.ctypes.data, nsel, None if s is None else s.ctypes.data, f.shape[1],
                                f.ctypes.data, k, kap.ctypes.data, leaf.ctypes.data, nf.ctypes.data,
                                nt.ctypes.data, nc.ctypes.data, lv.ctypes.data))
    out = (tuple(int(x) for x in kap[:n]), [int(x) for x in leaf])
    if not model:
        return out
    nleaves = int(leaf.max()) + 1 if leaf.size else 1
    nn = 2 * nleaves - 1
    return out + (nf[:nn].copy(), nt[:nn].copy(), nc[:2 * nn].copy(), [int(x) for x in lv[:nleaves]])


def ptune_tree_route(node_feat, node_thr, node_child, x):
    """Leaf index of feature vector x in a tree written by ptune_tree."""
    import numpy as np
    nf = np.ascontiguousarray(node_feat, dtype=np.int32)
    nt = np.ascontiguousarray(node_thr, dtype=np.float64)
    nc = np.ascontiguousarray(node_child, dtype=np.int32)
    xv = np.ascontiguousarray(x, dtype=np.float64)
    return _check(lib().ptune_tree_route(nf.size, nf.ctypes.data, nt.ctypes.data, nc.ctypes.data, xv.size,
                                         xv.ctypes.data))
