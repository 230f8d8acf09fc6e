"""Python binding of libsmx (the C ABI in include/smx.h).

Argument marshalling only: every step of the path (gather, Newton-Schulz
products, scatter, reductions) runs in the HIP kernels of libsmx.so.  The
library must have been built (``python paper_2004_10811_amd/build.py`` or
``__graft_entry__.build()``); importing this package without it raises.

PyTorch is optional here and only provides device memory and streams:
arrays may be numpy (host) or torch tensors (host or device).
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsmx.so")

SMX_OK = 0
SMX_E_INVALID = -1
SMX_E_STATE = -2
SMX_E_NOT_SYMMETRIC = -3
SMX_E_NONFINITE = -4
SMX_E_UNSUPPORTED = -5
SMX_E_NOMEM = -6
SMX_E_HIP = -7
SMX_E_NOT_CONVERGED = -8

SMX_FP64 = 0
SMX_BF16_3W = 1
SMX_BF16_1W = 2
SMX_FP32 = 3
SMX_FP16_2W = 4

SMX_SOLVER_ITERATIVE = 0
SMX_SOLVER_EIG = 1

SMX_ITER_NS2 = 0
SMX_ITER_PADE3 = 1
ITERATIONS = {"ns2": SMX_ITER_NS2, "pade3": SMX_ITER_PADE3}

PRECISIONS = {"fp64": SMX_FP64, "bf16x3": SMX_BF16_3W, "bf16": SMX_BF16_1W, "fp32": SMX_FP32,
              "fp16x2": SMX_FP16_2W}

# Every function the header declares, with (restype, argtypes).
_P = ctypes.POINTER
_i32, _i64, _f64, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class SmxStats(ctypes.Structure):
    _fields_ = [("ngroups", _i32), ("n_min", _i32), ("n_max", _i32), ("iters_min", _i32),
                ("iters_max", _i32), ("n_not_converged", _i32), ("precision", _i32), ("nwaves", _i32),
                ("n_mean", _f64), ("iters_mean", _f64), ("resid_max", _f64), ("algo_flops", _f64),
                ("exec_flops", _f64), ("time_gather_ms", _f64), ("time_iterate_ms", _f64),
                ("time_scatter_ms", _f64), ("time_total_ms", _f64), ("workspace_bytes", _f64)]


SIGNATURES = {
    "smx_create": (_i32, [_i32, _P(_vp)]),
    "smx_destroy": (_i32, [_vp]),
    "smx_last_error": (ctypes.c_char_p, [_vp]),
    "smx_set_stream": (_i32, [_vp, _vp]),
    "smx_load_k": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _i32]),
    "smx_update_values": (_i32, [_vp, _vp, _i32]),
    "smx_set_groups": (_i32, [_vp, _i32, _vp, _vp]),
    "smx_set_mu": (_i32, [_vp, _f64]),
    "smx_set_temperature": (_i32, [_vp, _f64]),
    "smx_set_precision": (_i32, [_vp, _i32]),
    "smx_set_convergence": (_i32, [_vp, _f64, _i32, _i32, _f64]),
    "smx_set_workspace_limit": (_i32, [_vp, _i64]),
    "smx_set_graph": (_i32, [_vp, _i32]),
    "smx_set_tile_order": (_i32, [_vp, _i32]),
    "smx_set_kernel_variant": (_i32, [_vp, _i32]),
    "smx_set_debug_checks": (_i32, [_vp, _i32]),
    "smx_set_tile_shape": (_i32, [_vp, _i32]),
    "smx_set_iteration": (_i32, [_vp, _i32]),
    "smx_set_solver": (_i32, [_vp, _i32]),
    "smx_group_speedup": (_i32, [_i32, _vp, _vp, _vp, _i32, _vp, _vp, _P(_f64), _P(_f64)]),
    "smx_group_kmeans": (_i32, [_i32, _vp, _f64, _i32, _i32, _i32, _P(_i32), _vp, _vp]),
    "smx_group_last_error": (ctypes.c_char_p, []),
    "smx_split_columns": (_i32, [_i32, _vp, _vp, _vp, _vp, _f64, _i32, _P(_i32), _P(_i64), _P(_i32), _vp, _vp,
                                 _vp, _vp, _vp, _vp]),
    "smx_get_d_expanded": (_i32, [_vp, _vp, _i64, _vp, _i32]),
    "smx_find_mu_eig": (_i32, [_vp, _f64, _f64, _i32, _P(_f64), _P(_i32)]),
    "smx_get_spectrum": (_i32, [_vp, _vp, _vp]),
    "smx_get_launch_config": (_i32, [_vp, _P(_i32), _P(_i32), _P(_i32), _P(_i32)]),
    "smx_autotune": (_i32, [_vp, _i32, _i32, _P(_i32), _P(_i32), _P(_f64)]),
    "smx_evaluate": (_i32, [_vp]),
    "smx_evaluate_static": (_i32, [_vp]),
    "smx_wait": (_i32, [_vp]),
    "smx_get_d": (_i32, [_vp, _vp, _i32]),
    "smx_trace": (_i32, [_vp, _P(_f64)]),
    "smx_energy": (_i32, [_vp, _P(_f64)]),
    "smx_get_stats": (_i32, [_vp, _P(SmxStats)]),
    "smx_get_group_info": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "smx_get_sizes": (_i32, [_vp, _P(_i32), _P(_i64)]),
    "smx_get_launch_profile": (_i32, [_vp, _i32, _vp, _vp, _vp, _P(_i32)]),
    "smx_get_launch_issued": (_i32, [_vp, _i32, _vp, _P(_i32)]),
    "smx_get_submatrix": (_i32, [_vp, _i32, _i32, _vp, _i32, _P(_i32)]),
    "smx_set_frozen": (_i32, [_vp, _i32]),
    "smx_dn_dmu": (_i32, [_vp, _P(_f64)]),
    "smx_find_mu": (_i32, [_vp, _f64, _f64, _i32, _P(_f64), _P(_i32)]),
    "smx_backward": (_i32, [_vp, _f64, _f64, _vp, _i32, _vp, _i32, _P(_f64)]),
    "smx_workspace_size": (_i32, [_vp, _P(ctypes.c_size_t)]),
    "smx_set_workspace": (_i32, [_vp, _vp, ctypes.c_size_t]),
    "smx_set_host_poll": (_i32, [_vp, _i32]),
    "smx_get_history": (_i32, [_vp, _i32, _vp, _vp, _vp]),
}

_lib = None


def _share_torch_hip_runtime():
    """Make libsmx bind to PyTorch's HIP runtime when PyTorch is installed.

    PyTorch ships its own libamdhip64 (same soname as the system one).  If the
    system copy were loaded first, a later ``import torch`` would bring in a
    second HIP runtime in the same process, and torch's streams and device
    pointers would not be valid for libsmx.  Loading torch's copy first (by
    path, without importing torch) makes every later load resolve to it.
    """
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec is None or not spec.submodule_search_locations:
            return
        for loc in spec.submodule_search_locations:
            p = os.path.join(loc, "lib", "libamdhip64.so")
            if os.path.exists(p):
                ctypes.CDLL(p, mode=ctypes.RTLD_GLOBAL)
                return
    except OSError:
        pass


def load_library(path: str = LIB_PATH):
    """Load libsmx.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"libsmx.so is not built ({path}); run __graft_entry__.build()")
        _share_torch_hip_runtime()
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class SmxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _ptr(a):
    """Raw address of a numpy array or torch tensor (host or device)."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())


def _on_device(a) -> int:
    return 0 if isinstance(a, np.ndarray) else int(getattr(a, "is_cuda", False))


# ---- thin wrappers with the C names ----------------------------------------

def _check(ctx, code):
    if code != SMX_OK:
        msg = load_library().smx_last_error(ctx).decode()
        raise SmxError(code, msg)
    return code


def smx_create(device: int = 0):
    lib = load_library()
    h = _vp()
    st = lib.smx_create(device, ctypes.byref(h))
    if st != SMX_OK:
        raise SmxError(st, lib.smx_last_error(None).decode())
    return h


def smx_destroy(ctx):
    return _check(ctx, load_library().smx_destroy(ctx))


def smx_set_stream(ctx, stream_handle: int):
    return _check(ctx, load_library().smx_set_stream(ctx, _vp(stream_handle)))


def smx_load_k(ctx, blk_size, col_ptr, row_idx, values):
    blk = np.ascontiguousarray(blk_size, dtype=np.int32)
    cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
    ri = np.ascontiguousarray(row_idx, dtype=np.int32)
    if isinstance(values, np.ndarray):
        values = np.ascontiguousarray(values, dtype=np.float64)
    return _check(ctx, load_library().smx_load_k(ctx, len(blk), blk.ctypes.data, cp.ctypes.data,
                                                  ri.ctypes.data, _ptr(values), _on_device(values)))


def smx_update_values(ctx, values):
    if isinstance(values, np.ndarray):
        values = np.ascontiguousarray(values, dtype=np.float64)
    return _check(ctx, load_library().smx_update_values(ctx, _ptr(values), _on_device(values)))


def smx_set_groups(ctx, grp_ptr, grp_blocks):
    gp = np.ascontiguousarray(grp_ptr, dtype=np.int32)
    gb = np.ascontiguousarray(grp_blocks, dtype=np.int32)
    return _check(ctx, load_library().smx_set_groups(ctx, len(gp) - 1, gp.ctypes.data, gb.ctypes.data))


def smx_set_mu(ctx, mu: float):
    return _check(ctx, load_library().smx_set_mu(ctx, float(mu)))


def smx_set_temperature(ctx, kT: float):
    return _check(ctx, load_library().smx_set_temperature(ctx, float(kT)))


def smx_set_precision(ctx, mode):
    if isinstance(mode, str):
        mode = PRECISIONS[mode]
    return _check(ctx, load_library().smx_set_precision(ctx, int(mode)))


def smx_set_convergence(ctx, tol=1e-12, max_iter=100, n_polish=2, switch_tol=1e-3):
    return _check(ctx, load_library().smx_set_convergence(ctx, float(tol), int(max_iter),
                                                           int(n_polish), float(switch_tol)))


def smx_set_workspace_limit(ctx, nbytes=0):
    return _check(ctx, load_library().smx_set_workspace_limit(ctx, int(nbytes)))


def smx_set_graph(ctx, steps_per_graph=0):
    return _check(ctx, load_library().smx_set_graph(ctx, int(steps_per_graph)))


def smx_set_tile_order(ctx, order=0):
    return _check(ctx, load_library().smx_set_tile_order(ctx, int(order)))


def smx_set_kernel_variant(ctx, variant=0):
    return _check(ctx, load_library().smx_set_kernel_variant(ctx, int(variant)))


def smx_set_debug_checks(ctx, on=True):
    return _check(ctx, load_library().smx_set_debug_checks(ctx, int(bool(on))))


def _group_check(st):
    if st != SMX_OK:
        raise SmxError(st, load_library().smx_group_last_error().decode())


def group_speedup(system, grp_ptr=None, grp_blocks=None):
    """(S, sum_g n_g^3) of Eq. estimatedspeedup for groups of the system's block
    columns (default: the system's own groups)."""
    gp = np.ascontiguousarray(system.grp_ptr if grp_ptr is None else grp_ptr, dtype=np.int32)
    gb = np.ascontiguousarray(system.grp_blocks if grp_blocks is None else grp_blocks, dtype=np.int32)
    bs = np.ascontiguousarray(system.blk_size, dtype=np.int32)
    cp = np.ascontiguousarray(system.col_ptr, dtype=np.int64)
    ri = np.ascontiguousarray(system.row_idx, dtype=np.int32)
    s, w = _f64(), _f64()
    _group_check(load_library().smx_group_speedup(int(len(bs)), bs.ctypes.data, cp.ctypes.data, ri.ctypes.data,
                                                  int(len(gp) - 1), gp.ctypes.data, gb.ctypes.data, ctypes.byref(s),
                                                  ctypes.byref(w)))
    return s.value, w.value


def group_kmeans(coords, nclusters, box=0.0, seed=0, max_iter=100):
    """(grp_ptr, grp_blocks): k-means clusters of the block columns' positions."""
    xyz = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 3)
    nb = xyz.shape[0]
    gp = np.zeros(int(nclusters) + 1, np.int32)
    gb = np.zeros(nb, np.int32)
    ng = _i32()
    _group_check(load_library().smx_group_kmeans(int(nb), xyz.ctypes.data, float(box), int(nclusters), int(seed),
                                                 int(max_iter), ctypes.byref(ng), gp.ctypes.data, gb.ctypes.data))
    return gp[:ng.value + 1].copy(), gb


@dataclass
class SplitProblem:
    """The element-level problem of smx_split_columns (the BSC fields Context.load
    reads) and src, the position of each of its values in the block layout."""
    blk_size: np.ndarray
    col_ptr: np.ndarray
    row_idx: np.ndarray
    values: np.ndarray
    grp_ptr: np.ndarray
    grp_blocks: np.ndarray
    mu: float
    src: np.ndarray
    nvalues_block: int


def split_columns(system, eps, merge=True):
    """Sub-submatrices of single columns (smx_split_columns) as a SplitProblem."""
    bs = np.ascontiguousarray(system.blk_size, dtype=np.int32)
    cp = np.ascontiguousarray(system.col_ptr, dtype=np.int64)
    ri = np.ascontiguousarray(system.row_idx, dtype=np.int32)
    vals = np.ascontiguousarray(system.values, dtype=np.float64)
    n, nnz, ng = _i32(), _i64(), _i32()
    lib = load_library()
    _group_check(lib.smx_split_columns(len(bs), bs.ctypes.data, cp.ctypes.data, ri.ctypes.data, vals.ctypes.data,
                                       float(eps), int(bool(merge)), ctypes.byref(n), ctypes.byref(nnz),
                                       ctypes.byref(ng), None, None, None, None, None, None))
    ecp = np.zeros(n.value + 1, np.int64)
    eri = np.zeros(nnz.value, np.int32)
    ev = np.zeros(nnz.value)
    es = np.zeros(nnz.value, np.int64)
    egp = np.zeros(ng.value + 1, np.int32)
    egc = np.zeros(n.value, np.int32)
    _group_check(lib.smx_split_columns(len(bs), bs.ctypes.data, cp.ctypes.data, ri.ctypes.data, vals.ctypes.data,
                                       float(eps), int(bool(merge)), ctypes.byref(n), ctypes.byref(nnz),
                                       ctypes.byref(ng), ecp.ctypes.data, eri.ctypes.data, ev.ctypes.data,
                                       es.ctypes.data, egp.ctypes.data, egc.ctypes.data))
    return SplitProblem(np.ones(n.value, np.int32), ecp, eri, ev, egp, egc, float(system.mu), es, len(vals))


def smx_get_d_expanded(ctx, index, n_out, out=None):
    """D of the last evaluation in another layout: out[index[q]] = D_q, 0 elsewhere."""
    idx = np.ascontiguousarray(index, dtype=np.int64)
    if out is None:
        out = np.empty(int(n_out))
    _check(ctx, load_library().smx_get_d_expanded(ctx, idx.ctypes.data, int(n_out), _ptr(out), _on_device(out)))
    return out


def smx_set_solver(ctx, solver="iterative"):
    k = {"iterative": SMX_SOLVER_ITERATIVE, "eig": SMX_SOLVER_EIG}[solver] if isinstance(solver, str) else int(solver)
    return _check(ctx, load_library().smx_set_solver(ctx, k))


def smx_find_mu_eig(ctx, n_target: float, tol: float = 1e-8, max_steps: int = 20, allow_not_converged=False):
    """(mu, bisection steps, status): Algorithm 1 on the stored decompositions."""
    mu, steps = _f64(), _i32()
    st = load_library().smx_find_mu_eig(ctx, float(n_target), float(tol), int(max_steps), ctypes.byref(mu),
                                        ctypes.byref(steps))
    if not (allow_not_converged and st == SMX_E_NOT_CONVERGED):
        _check(ctx, st)
    return mu.value, steps.value, st


def smx_get_spectrum(ctx):
    """(eigenvalues, weights) of every group's submatrix, concatenated by group."""
    ng, _ = smx_get_sizes(ctx)
    info = smx_get_group_info(ctx)
    tot = int(info["n"].sum())
    lam = np.zeros(tot)
    w = np.zeros(tot)
    _check(ctx, load_library().smx_get_spectrum(ctx, lam.ctypes.data, w.ctypes.data))
    return lam, w


def smx_set_iteration(ctx, kind="ns2"):
    k = ITERATIONS[kind] if isinstance(kind, str) else int(kind)
    return _check(ctx, load_library().smx_set_iteration(ctx, k))


def smx_set_tile_shape(ctx, big_min_npad=0):
    return _check(ctx, load_library().smx_set_tile_shape(ctx, int(big_min_npad)))


def smx_get_launch_config(ctx) -> dict:
    g, o, b, v = _i32(), _i32(), _i32(), _i32()
    _check(ctx, load_library().smx_get_launch_config(ctx, ctypes.byref(g), ctypes.byref(o), ctypes.byref(b),
                                                     ctypes.byref(v)))
    return dict(graph_steps=g.value, tile_order=o.value, big_min_npad=b.value, kernel_variant=v.value)


def smx_autotune(ctx, reps=3, use_cache=True):
    """Time the candidate launch configurations; returns (graph_steps, tile_order, best_ms)."""
    g, o, ms = _i32(), _i32(), _f64()
    _check(ctx, load_library().smx_autotune(ctx, int(reps), int(bool(use_cache)), ctypes.byref(g),
                                            ctypes.byref(o), ctypes.byref(ms)))
    return g.value, o.value, ms.value


def smx_evaluate(ctx):
    return _check(ctx, load_library().smx_evaluate(ctx))


def smx_evaluate_static(ctx):
    return _check(ctx, load_library().smx_evaluate_static(ctx))


def smx_wait(ctx, allow_not_converged: bool = False):
    st = load_library().smx_wait(ctx)
    if allow_not_converged and st == SMX_E_NOT_CONVERGED:
        return st
    return _check(ctx, st)


def smx_get_d(ctx, out):
    return _check(ctx, load_library().smx_get_d(ctx, _ptr(out), _on_device(out)))


def smx_trace(ctx) -> float:
    v = _f64()
    _check(ctx, load_library().smx_trace(ctx, ctypes.byref(v)))
    return v.value


def smx_energy(ctx) -> float:
    v = _f64()
    _check(ctx, load_library().smx_energy(ctx, ctypes.byref(v)))
    return v.value


def smx_get_stats(ctx) -> dict:
    s = SmxStats()
    _check(ctx, load_library().smx_get_stats(ctx, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in SmxStats._fields_}


def smx_get_sizes(ctx):
    ng, nv = _i32(), _i64()
    _check(ctx, load_library().smx_get_sizes(ctx, ctypes.byref(ng), ctypes.byref(nv)))
    return ng.value, nv.value


def smx_get_group_info(ctx):
    ng, _ = smx_get_sizes(ctx)
    n = np.zeros(ng, np.int32)
    it = np.zeros(ng, np.int32)
    sc = np.zeros(ng)
    rs = np.zeros(ng)
    _check(ctx, load_library().smx_get_group_info(ctx, n.ctypes.data, it.ctypes.data,
                                                   sc.ctypes.data, rs.ctypes.data))
    return dict(n=n, iters=it, scale=sc, resid=rs)


def smx_get_launch_profile(ctx):
    """(ms, algorithmic flops, kind) per product-kernel launch of the last evaluation."""
    cnt = _i32()
    _check(ctx, load_library().smx_get_launch_profile(ctx, 0, None, None, None, ctypes.byref(cnt)))
    n = cnt.value
    ms = np.zeros(n, np.float32)
    fl = np.zeros(n)
    kd = np.zeros(n, np.int32)
    _check(ctx, load_library().smx_get_launch_profile(ctx, n, ms.ctypes.data, fl.ctypes.data,
                                                       kd.ctypes.data, ctypes.byref(cnt)))
    return ms.astype(np.float64), fl, kd


def smx_get_launch_issued(ctx):
    """Issued matrix-core flops per product-kernel launch (order of smx_get_launch_profile)."""
    cnt = _i32()
    _check(ctx, load_library().smx_get_launch_issued(ctx, 0, None, ctypes.byref(cnt)))
    out = np.zeros(cnt.value)
    _check(ctx, load_library().smx_get_launch_issued(ctx, cnt.value, out.ctypes.data, ctypes.byref(cnt)))
    return out


def smx_get_submatrix(ctx, g: int, what: int = 1) -> np.ndarray:
    """Group g's dense submatrix: what=0 the gathered A_g, what=1 its sign S_g."""
    n = _i32()
    _check(ctx, load_library().smx_get_submatrix(ctx, g, what, None, 0, ctypes.byref(n)))
    out = np.zeros((n.value, n.value), order="F")
    _check(ctx, load_library().smx_get_submatrix(ctx, g, what, out.ctypes.data, max(n.value, 1),
                                                  ctypes.byref(n)))
    return np.ascontiguousarray(out)


def smx_set_frozen(ctx, on: bool = True):
    return _check(ctx, load_library().smx_set_frozen(ctx, int(bool(on))))


def smx_dn_dmu(ctx) -> float:
    v = _f64()
    _check(ctx, load_library().smx_dn_dmu(ctx, ctypes.byref(v)))
    return v.value


def smx_find_mu(ctx, n_target: float, tol: float = 1e-8, max_steps: int = 50):
    """(mu, evaluations used) with N(mu) = n_target on the frozen iteration."""
    mu, steps = _f64(), _i32()
    _check(ctx, load_library().smx_find_mu(ctx, float(n_target), float(tol), int(max_steps),
                                            ctypes.byref(mu), ctypes.byref(steps)))
    return mu.value, steps.value


def smx_backward(ctx, gE: float = 0.0, gN: float = 0.0, gD=None, out=None):
    """(dL/dK in K's layout, dL/dmu) for L = gE E + gN N + <gD, D> on the frozen last evaluation."""
    if gD is not None and isinstance(gD, np.ndarray):
        gD = np.ascontiguousarray(gD, dtype=np.float64)
    if out is None:
        _, nv = smx_get_sizes(ctx)
        out = np.empty(nv)
    dmu = _f64()
    _check(ctx, load_library().smx_backward(ctx, float(gE), float(gN),
                                             None if gD is None else _ptr(gD),
                                             0 if gD is None else _on_device(gD),
                                             _ptr(out), _on_device(out), ctypes.byref(dmu)))
    return out, dmu.value


def smx_workspace_size(ctx) -> int:
    """Bytes of a work space holding every submatrix at once."""
    v = ctypes.c_size_t()
    _check(ctx, load_library().smx_workspace_size(ctx, ctypes.byref(v)))
    return v.value


def smx_set_workspace(ctx, buf=None, nbytes=None):
    """Use device memory `buf` (a torch tensor, or a raw device address with
    `nbytes`) as the evaluation work space; None returns to library memory."""
    if buf is None:
        return _check(ctx, load_library().smx_set_workspace(ctx, None, 0))
    if nbytes is None:
        nbytes = buf.numel() * buf.element_size()
    return _check(ctx, load_library().smx_set_workspace(ctx, _vp(_ptr(buf) if not isinstance(buf, int) else buf),
                                                         int(nbytes)))


def smx_set_host_poll(ctx, on: bool = True):
    return _check(ctx, load_library().smx_set_host_poll(ctx, int(bool(on))))


def smx_get_history(ctx, cap: int = 128):
    """Per-group histories of the last evaluation: dict(resid, tau) of shape
    (ngroups, cap) (NaN past each group's steps) and nsteps (ngroups,)."""
    ng, _ = smx_get_sizes(ctx)
    r = np.zeros((ng, cap))
    t = np.zeros((ng, cap))
    n = np.zeros(ng, np.int32)
    _check(ctx, load_library().smx_get_history(ctx, int(cap), r.ctypes.data, t.ctypes.data, n.ctypes.data))
    return dict(resid=r, tau=t, nsteps=n)


# ---- convenience object -----------------------------------------------------

@dataclass
class Result:
    d_values: object
    n_elec: float
    energy: float
    status: int


class Context:
    """Owns one smx context; `system` is any object with the BSC fields
    (blk_size, col_ptr, row_idx, values, grp_ptr, grp_blocks, mu)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.handle = smx_create(device)
        if stream is not None:
            smx_set_stream(self.handle, stream)
        self.nvalues = 0

    def close(self):
        if self.handle is not None:
            smx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, system, values=None):
        vals = system.values if values is None else values
        smx_load_k(self.handle, system.blk_size, system.col_ptr, system.row_idx, vals)
        smx_set_groups(self.handle, system.grp_ptr, system.grp_blocks)
        smx_set_mu(self.handle, getattr(system, "mu", 0.0))
        _, self.nvalues = smx_get_sizes(self.handle)
        return self

    def configure(self, precision="fp64", tol=1e-12, max_iter=100, n_polish=2, switch_tol=1e-3,
                  mu=None, kT=None, workspace_limit=None, graph_steps=None, tile_shape=None, iteration=None,
                  solver=None):
        smx_set_precision(self.handle, precision)
        if solver is not None:
            smx_set_solver(self.handle, solver)
        if iteration is not None:
            smx_set_iteration(self.handle, iteration)
        if tile_shape is not None:
            smx_set_tile_shape(self.handle, tile_shape)
        if graph_steps is not None:
            smx_set_graph(self.handle, graph_steps)
        if workspace_limit is not None:
            smx_set_workspace_limit(self.handle, workspace_limit)
        smx_set_convergence(self.handle, tol, max_iter, n_polish, switch_tol)
        if mu is not None:
            smx_set_mu(self.handle, mu)
        if kT is not None:
            smx_set_temperature(self.handle, kT)
        return self

    def evaluate(self, out=None, allow_not_converged=False) -> Result:
        smx_evaluate(self.handle)
        st = smx_wait(self.handle, allow_not_converged)
        if out is None:
            out = np.empty(self.nvalues)
        smx_get_d(self.handle, out)
        return Result(out, smx_trace(self.handle), smx_energy(self.handle), st)

    def evaluate_static(self, out=None, allow_not_converged=False) -> Result:
        """smx_evaluate_static: the same evaluation with all work memory in the
        library's fixed scratch array (no allocation inside the call)."""
        smx_evaluate_static(self.handle)
        st = smx_wait(self.handle, allow_not_converged)
        if out is None:
            out = np.empty(self.nvalues)
        smx_get_d(self.handle, out)
        return Result(out, smx_trace(self.handle), smx_energy(self.handle), st)

    def stats(self) -> dict:
        return smx_get_stats(self.handle)

    def group_info(self) -> dict:
        return smx_get_group_info(self.handle)

    def submatrix(self, g: int, what: int = 1) -> np.ndarray:
        return smx_get_submatrix(self.handle, g, what)

    def launch_profile(self):
        return smx_get_launch_profile(self.handle)

    def backward(self, gE=0.0, gN=0.0, gD=None, out=None):
        return smx_backward(self.handle, gE, gN, gD, out)


def submatrix_sign_function():
    """torch.autograd.Function mapping (K values, mu) -> (D values, N, E).

    Forward: one evaluation of the hot path (any precision mode of the
    context).  Backward: the hand-written adjoint (smx_backward) of the frozen
    Newton-Schulz map of that evaluation, returning (dK, dmu).  Built lazily so
    the binding does not need torch.
    """
    import torch

    class SubmatrixSign(torch.autograd.Function):
        @staticmethod
        def forward(fctx, kvals, mu, holder):
            c = holder.ctx
            smx_update_values(c.handle, kvals.detach().contiguous())
            smx_set_mu(c.handle, float(mu))
            d = torch.empty_like(kvals)
            r = c.evaluate(out=d)
            holder.token += 1
            fctx.holder = holder
            fctx.token = holder.token
            fctx.save_for_backward(kvals, mu if torch.is_tensor(mu) else torch.tensor(float(mu)))
            dev = kvals.device
            return d, torch.tensor(r.n_elec, dtype=torch.float64, device=dev), \
                torch.tensor(r.energy, dtype=torch.float64, device=dev)

        @staticmethod
        def backward(fctx, gD, gN, gE):
            holder = fctx.holder
            c = holder.ctx
            kvals, mu = fctx.saved_tensors
            if holder.token != fctx.token:
                # another evaluation ran in between: restore this one's state
                smx_update_values(c.handle, kvals.detach().contiguous())
                smx_set_mu(c.handle, float(mu))
                c.evaluate(out=torch.empty_like(kvals))
                holder.token += 1
            ge = 0.0 if gE is None else float(gE)
            gn = 0.0 if gN is None else float(gN)
            gd = None if gD is None else gD.detach().contiguous().to(torch.float64)
            dk = torch.empty_like(kvals)
            _, dmu = smx_backward(c.handle, ge, gn, gd, dk)
            gmu = torch.tensor(dmu, dtype=torch.float64, device=mu.device) if fctx.needs_input_grad[1] else None
            return (dk if fctx.needs_input_grad[0] else None), gmu, None

    return SubmatrixSign


class SubmatrixSign:
    """Differentiable (K values, mu) -> (D values, N, E) on one context.

    ``SubmatrixSign(ctx)(kvals, mu)`` with ``kvals`` a CUDA float64 tensor in
    the layout loaded into ``ctx`` (``ctx.load(system)`` first).
    """

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.token = 0
        self._fn = submatrix_sign_function()

    def __call__(self, kvals, mu):
        return self._fn.apply(kvals, mu, self)
