"""ctypes binding of libfill.so (the C ABI declared in include/fill.h).

Argument marshalling only: every step of the fill runs in the HIP kernels of
the library.  The functions keep the C names; `Plan` is a small owner of a
fill_plan handle that passes torch tensors' device pointers and the current
HIP stream through.  If the library is missing this module raises at import:
there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FILL_LIBRARY may name another build of the same library (the FFT autotuner
# loads its candidate builds this way); by default the in-tree build.
LIB_PATH = os.environ.get("FILL_LIBRARY") or os.path.join(HERE, "libfill.so")

FILL_OK = 0
FILL_EINVAL = -1
FILL_ENOMEM = -2
FILL_EHIP = -3
FILL_ENOCONV = -4
FILL_EUNSUPPORTED_SIZE = -5
FILL_ENOTSPD = -6

FILL_PREC_FP64 = 0
FILL_PREC_FP32_OP = 1

FILL_OP_CINV = 0
FILL_OP_CHALF = 1
FILL_OP_A = 2
FILL_OP_E = 3
FILL_OP_MINV = 4

# every symbol include/fill.h declares
EXPORTS = (
    "fill_supported_size", "fill_plan_create", "fill_plan_create_batch", "fill_plan_nprob",
    "fill_plan_set_pk", "fill_plan_set_max_iter", "fill_plan_set_inner_tol", "fill_realize_batch",
    "fill_mean_batch", "fill_realize_multi", "fill_get_stats_batch", "fill_plan_set_bands",
    "fill_adjoint", "fill_adjoint_batch",
    "fill_plan_destroy", "fill_realize", "fill_mean", "fill_get_stats", "fill_apply",
    "fill_realize_unconstrained", "fill_philox_words", "fill_time_kernel", "fill_kernel_timing",
    "fill_kernel_timing_read", "fill_strerror",
    "fill_last_error", "fill_plan_set_precond", "fill_plan_set_lanczos", "fill_get_lanczos",
    "fill_lanczos_extremes", "fill_plan_set_graph", "fill_plan_set_skew", "fill_strips_create",
    "fill_strips_mean", "fill_strips_mask", "fill_strips_plan", "fill_strips_last_error", "fill_strips_destroy",
    "fill_strips_refine", "fill_laplace", "fill_plan_set_cg", "fill_get_block_info",
    "fill_realize_unconstrained_noalloc", "fill_group_create", "fill_group_realize", "fill_group_last_graph",
    "fill_group_destroy", "fill_plan_set_warm_start", "fill_plan_set_block_halo",
)

FILL_PRECOND_NONE = 0
FILL_PRECOND_SPLIT = 1
FILL_PRECOND_CXX = 2
FILL_PRECOND_BLOCK = 3
FILL_BLOCK_HALO_AUTO = -1

FILL_CG_STANDARD = 0
FILL_CG_SINGLE_REDUCTION = 1

FILL_K_R2C = 0
FILL_K_COL = 1
FILL_K_C2R = 2
FILL_K_APPLY = 3
FILL_K_PROJ = 4
FILL_K_BAND = 5
FILL_K_BLOCKMV = 6
FILL_K_COMBINE = 7


class fill_stats(C.Structure):
    _fields_ = [("iters_inner", C.c_int), ("iters_outer", C.c_int), ("n_masked", C.c_int),
                ("status", C.c_int), ("rel_resid", C.c_double), ("solve_ms", C.c_double),
                ("whole_graph", C.c_int)]


class BlockInfo(C.Structure):
    _fields_ = [("runs", C.c_int), ("blocks", C.c_int), ("band_rows", C.c_int64), ("block_pixels", C.c_int64),
                ("block_entries", C.c_int64), ("bytes", C.c_int64), ("elem_bytes", C.c_int),
                ("band_stream_values", C.c_int64), ("halo_min", C.c_int), ("halo_max", C.c_int)]


class FillError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {_strerror(code)} ({code}): {detail}")
        self.code = code


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1109_0286_amd/build.py`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, u64, dbl = C.c_void_p, C.c_int, C.c_uint64, C.c_double
    sig = {
        "fill_supported_size": (i32, [i32]),
        "fill_plan_create": (i32, [i32, i32, vp, vp, i32, vp, C.POINTER(vp)]),
        "fill_plan_create_batch": (i32, [i32, i32, i32, vp, vp, i32, i32, vp, C.POINTER(vp)]),
        "fill_plan_nprob": (i32, [vp]),
        "fill_realize_batch": (i32, [vp, vp, vp, vp, dbl]),
        "fill_mean_batch": (i32, [vp, vp, vp, dbl]),
        "fill_realize_multi": (i32, [i32, vp, vp, vp, vp, dbl]),
        "fill_group_create": (i32, [i32, vp, vp, C.POINTER(vp)]),
        "fill_group_realize": (i32, [vp, vp, vp, vp, dbl]),
        "fill_group_last_graph": (i32, [vp]),
        "fill_group_destroy": (None, [vp]),
        "fill_get_stats_batch": (i32, [vp, C.POINTER(fill_stats)]),
        "fill_plan_set_bands": (i32, [vp, i32, vp, vp]),
        "fill_adjoint": (i32, [vp, vp, u64, vp, vp, vp, vp, vp, dbl]),
        "fill_adjoint_batch": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, dbl]),
        "fill_plan_set_pk": (i32, [vp, vp]),
        "fill_plan_set_max_iter": (i32, [vp, i32]),
        "fill_plan_set_inner_tol": (i32, [vp, dbl]),
        "fill_plan_set_precond": (i32, [vp, i32]),
        "fill_plan_set_block_halo": (i32, [vp, i32]),
        "fill_plan_set_cg": (i32, [vp, i32]),
        "fill_get_block_info": (i32, [vp, C.POINTER(BlockInfo)]),
        "fill_plan_set_graph": (i32, [vp, i32]),
        "fill_plan_set_skew": (i32, [vp, dbl]),
        "fill_strips_create": (i32, [i32, i32, vp, vp, dbl, i32, vp, vp, dbl, i32, i32, vp, C.POINTER(vp)]),
        "fill_strips_mean": (i32, [vp, vp, vp]),
        "fill_strips_refine": (i32, [vp, vp]),
        "fill_laplace": (i32, [vp, vp, vp, i32, dbl, dbl, i32]),
        "fill_plan_set_warm_start": (i32, [vp, i32, i32, dbl, dbl]),
        "fill_strips_mask": (i32, [vp, i32, vp]),
        "fill_strips_plan": (i32, [vp, i32, C.POINTER(vp)]),
        "fill_strips_last_error": (C.c_char_p, []),
        "fill_strips_destroy": (None, [vp]),
        "fill_plan_set_lanczos": (i32, [vp, i32]),
        "fill_get_lanczos": (i32, [vp, i32, vp, vp, i32, C.POINTER(i32)]),
        "fill_lanczos_extremes": (i32, [vp, i32, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(i32)]),
        "fill_plan_destroy": (None, [vp]),
        "fill_realize": (i32, [vp, vp, u64, vp, dbl]),
        "fill_mean": (i32, [vp, vp, vp, dbl]),
        "fill_get_stats": (i32, [vp, C.POINTER(fill_stats)]),
        "fill_apply": (i32, [vp, i32, i32, vp, vp]),
        "fill_realize_unconstrained": (i32, [vp, u64, vp]),
        "fill_realize_unconstrained_noalloc": (i32, [vp, u64, vp]),
        "fill_philox_words": (i32, [u64, u64, C.c_int64, vp]),
        "fill_time_kernel": (i32, [vp, i32, i32, i32, C.POINTER(dbl)]),
        "fill_kernel_timing": (i32, [vp, i32, i32]),
        "fill_kernel_timing_read": (i32, [vp, C.POINTER(dbl), C.POINTER(C.c_int64)]),
        "fill_strerror": (C.c_char_p, [i32]),
        "fill_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _strerror(code: int) -> str:
    return _lib.fill_strerror(code).decode()


def _check(code: int, where: str, ok=(FILL_OK,)) -> int:
    if code not in ok:
        raise FillError(code, where, _lib.fill_last_error().decode())
    return code


# ---- raw C names -----------------------------------------------------------

def fill_supported_size(n: int) -> bool:
    return bool(_lib.fill_supported_size(int(n)))


def fill_plan_create(nx, ny, mask, Pk, prec, stream) -> int:
    """mask: host uint8 (ny, nx); Pk: host float64 (ny, nx//2+1); stream: int handle or None."""
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    p = np.ascontiguousarray(Pk, dtype=np.float64)
    if m.shape != (ny, nx) or p.shape != (ny, nx // 2 + 1):
        raise ValueError(f"mask {m.shape} / Pk {p.shape} do not match grid {nx}x{ny}")
    h = C.c_void_p()
    _check(_lib.fill_plan_create(nx, ny, m.ctypes.data, p.ctypes.data, prec, stream or None, C.byref(h)),
           "fill_plan_create")
    return h.value


def fill_plan_create_batch(nx, ny, masks, Pk, prec, stream) -> int:
    """masks: host uint8 (nprob, ny, nx); Pk: host float64 (ny, nx//2+1) shared or (nprob, ny, nx//2+1)."""
    m = np.ascontiguousarray(masks, dtype=np.uint8)
    p = np.ascontiguousarray(Pk, dtype=np.float64)
    if m.ndim != 3 or m.shape[1:] != (ny, nx):
        raise ValueError(f"masks {m.shape} do not match grid {nx}x{ny}")
    nprob = m.shape[0]
    if p.shape == (ny, nx // 2 + 1):
        npk = 1
    elif p.shape == (nprob, ny, nx // 2 + 1):
        npk = nprob
    else:
        raise ValueError(f"Pk {p.shape} is neither one table nor one per problem")
    h = C.c_void_p()
    _check(_lib.fill_plan_create_batch(nx, ny, nprob, m.ctypes.data, p.ctypes.data, npk, prec, stream or None,
                                       C.byref(h)), "fill_plan_create_batch")
    return h.value


def fill_plan_nprob(plan) -> int:
    return _lib.fill_plan_nprob(plan)


def _ptr_array(ptrs):
    return (C.c_void_p * len(ptrs))(*ptrs)


def fill_realize_batch(plan, d_ptrs, seeds, x_ptrs, rtol, allow_noconv=False):
    ok = (FILL_OK, FILL_ENOCONV) if allow_noconv else (FILL_OK,)
    s = (C.c_uint64 * len(seeds))(*[int(v) for v in seeds])
    return _check(_lib.fill_realize_batch(plan, _ptr_array(d_ptrs), s, _ptr_array(x_ptrs), float(rtol)),
                  "fill_realize_batch", ok)


def fill_mean_batch(plan, d_ptrs, x_ptrs, rtol, allow_noconv=False):
    ok = (FILL_OK, FILL_ENOCONV) if allow_noconv else (FILL_OK,)
    return _check(_lib.fill_mean_batch(plan, _ptr_array(d_ptrs), _ptr_array(x_ptrs), float(rtol)),
                  "fill_mean_batch", ok)


def fill_realize_multi(plans, d_ptrs, seeds, x_ptrs, rtol, allow_noconv=False):
    """plans: list of handles; d_ptrs/x_ptrs/seeds: per plan, one entry per problem."""
    ok = (FILL_OK, FILL_ENOCONV) if allow_noconv else (FILL_OK,)
    n = len(plans)
    keep = []
    dd = (C.c_void_p * n)()
    xx = (C.c_void_p * n)()
    ss = (C.c_void_p * n)()
    for i in range(n):
        a, x = _ptr_array(d_ptrs[i]), _ptr_array(x_ptrs[i])
        s = (C.c_uint64 * len(seeds[i]))(*[int(v) for v in seeds[i]])
        keep += [a, x, s]
        dd[i] = C.cast(a, C.c_void_p)
        xx[i] = C.cast(x, C.c_void_p)
        ss[i] = C.cast(s, C.c_void_p)
    return _check(_lib.fill_realize_multi(n, _ptr_array(plans), dd, ss, xx, float(rtol)), "fill_realize_multi", ok)


def _plan_arrays(d_ptrs, seeds, x_ptrs):
    """Per-plan host arrays of device pointers and seeds (and what keeps them alive)."""
    n = len(d_ptrs)
    keep = []
    dd = (C.c_void_p * n)()
    xx = (C.c_void_p * n)()
    ss = (C.c_void_p * n)()
    for i in range(n):
        a, x = _ptr_array(d_ptrs[i]), _ptr_array(x_ptrs[i])
        s = (C.c_uint64 * len(seeds[i]))(*[int(v) for v in seeds[i]])
        keep += [a, x, s]
        dd[i] = C.cast(a, C.c_void_p)
        xx[i] = C.cast(x, C.c_void_p)
        ss[i] = C.cast(s, C.c_void_p)
    return dd, ss, xx, keep


def fill_group_create(plans, stream) -> int:
    out = C.c_void_p()
    _check(_lib.fill_group_create(len(plans), _ptr_array(plans), stream, C.byref(out)), "fill_group_create")
    return out.value


def fill_group_realize(group, d_ptrs, seeds, x_ptrs, rtol, allow_noconv=False):
    """d_ptrs/x_ptrs/seeds: per plan of the group, one entry per problem."""
    ok = (FILL_OK, FILL_ENOCONV) if allow_noconv else (FILL_OK,)
    dd, ss, xx, _keep = _plan_arrays(d_ptrs, seeds, x_ptrs)
    return _check(_lib.fill_group_realize(group, dd, ss, xx, float(rtol)), "fill_group_realize", ok)


def fill_group_last_graph(group) -> bool:
    return bool(_lib.fill_group_last_graph(group))


def fill_group_destroy(group):
    _lib.fill_group_destroy(group)


def fill_get_stats_batch(plan) -> list:
    n = fill_plan_nprob(plan)
    arr = (fill_stats * n)()
    _check(_lib.fill_get_stats_batch(plan, arr), "fill_get_stats_batch")
    return [{k: getattr(s, k) for k, _ in fill_stats._fields_} for s in arr]


def fill_plan_set_bands(plan, lnk_nodes, theta):
    lnk = np.ascontiguousarray(lnk_nodes, dtype=np.float64)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if lnk.shape != th.shape or lnk.ndim != 1:
        raise ValueError("lnk_nodes and theta must be 1-D of the same length")
    return _check(_lib.fill_plan_set_bands(plan, len(lnk), lnk.ctypes.data, th.ctypes.data), "fill_plan_set_bands")


def fill_adjoint_batch(plan, d_ptrs, seeds, x_ptrs, g_ptrs, gy_ptrs, nbands, nt=None, rtol=1e-10,
                       want_logP=False, allow_noconv=False):
    """Returns (grad_theta or None, grad_logP or None) as numpy arrays."""
    ok = (FILL_OK, FILL_ENOCONV) if allow_noconv else (FILL_OK,)
    s = (C.c_uint64 * len(seeds))(*[int(v) for v in seeds])
    gth = np.zeros(nbands) if nbands else None
    glp = np.zeros(len(d_ptrs) * nt) if want_logP else None
    _check(_lib.fill_adjoint_batch(plan, _ptr_array(d_ptrs), s, _ptr_array(x_ptrs), _ptr_array(g_ptrs),
                                   _ptr_array(gy_ptrs), gth.ctypes.data if gth is not None else None,
                                   glp.ctypes.data if glp is not None else None, float(rtol)),
           "fill_adjoint_batch", ok)
    return gth, glp


def fill_plan_set_pk(plan, Pk):
    p = np.ascontiguousarray(Pk, dtype=np.float64)
    return _check(_lib.fill_plan_set_pk(plan, p.ctypes.data), "fill_plan_set_pk")


def fill_plan_set_max_iter(plan, max_iter):
    return _check(_lib.fill_plan_set_max_iter(plan, int(max_iter)), "fill_plan_set_max_iter")


def fill_plan_set_inner_tol(plan, tol):
    return _check(_lib.fill_plan_set_inner_tol(plan, float(tol)), "fill_plan_set_inner_tol")


def fill_plan_set_precond(plan, mode):
    """mode: FILL_PRECOND_NONE / _SPLIT / _CXX / _BLOCK (True/False map to SPLIT/NONE)."""
    if mode is True or mode is False:
        mode = FILL_PRECOND_SPLIT if mode else FILL_PRECOND_NONE
    return _check(_lib.fill_plan_set_precond(plan, int(mode)), "fill_plan_set_precond")


def fill_plan_set_block_halo(plan, halo):
    """halo: 0..14, or FILL_BLOCK_HALO_AUTO (the default: per problem, from 8
    up by 2 while the dense blocks gain at most nx*ny/2 inverse entries)."""
    return _check(_lib.fill_plan_set_block_halo(plan, int(halo)), "fill_plan_set_block_halo")


def fill_get_block_info(plan) -> dict:
    """Runs, blocks, padded band rows, block pixels, inverse entries, bytes,
    element size, stored band factor values and the blocks' halos of the
    plan's block preconditioner."""
    out = BlockInfo()
    _check(_lib.fill_get_block_info(plan, C.byref(out)), "fill_get_block_info")
    return {f: getattr(out, f) for f, _ in BlockInfo._fields_}


def fill_plan_set_cg(plan, variant):
    """variant: FILL_CG_STANDARD or FILL_CG_SINGLE_REDUCTION."""
    return _check(_lib.fill_plan_set_cg(plan, int(variant)), "fill_plan_set_cg")


def fill_plan_set_warm_start(plan, iters, nkernels=8, r0=1.5, ratio=2.0):
    return _check(_lib.fill_plan_set_warm_start(plan, int(iters), int(nkernels), float(r0), float(ratio)),
                  "fill_plan_set_warm_start")


def fill_plan_set_skew(plan, eps):
    return _check(_lib.fill_plan_set_skew(plan, float(eps)), "fill_plan_set_skew")


def fill_plan_set_graph(plan, on):
    return _check(_lib.fill_plan_set_graph(plan, 1 if on else 0), "fill_plan_set_graph")


def fill_plan_set_lanczos(plan, cap):
    return _check(_lib.fill_plan_set_lanczos(plan, int(cap)), "fill_plan_set_lanczos")


def fill_get_lanczos(plan, problem, cap):
    """(alpha[k], beta[k-1]) recorded for one problem, k = min(steps, cap)."""
    al = np.zeros(max(int(cap), 1))
    be = np.zeros(max(int(cap), 1))
    n = C.c_int(0)
    _check(_lib.fill_get_lanczos(plan, int(problem), al.ctypes.data, be.ctypes.data, int(cap), C.byref(n)),
           "fill_get_lanczos")
    k = min(n.value, int(cap))
    return al[:k].copy(), be[:max(k - 1, 0)].copy()


def fill_lanczos_extremes(plan, problem):
    """(lambda_min, lambda_max, steps) of the recorded Lanczos matrix."""
    lo, hi, n = C.c_double(0.0), C.c_double(0.0), C.c_int(0)
    _check(_lib.fill_lanczos_extremes(plan, int(problem), C.byref(lo), C.byref(hi), C.byref(n)),
           "fill_lanczos_extremes")
    return lo.value, hi.value, n.value


def fill_plan_destroy(plan):
    _lib.fill_plan_destroy(plan)


def fill_realize(plan, d_obs_ptr, seed, x_out_ptr, rtol, allow_noconv=False):
    ok = (FILL_OK, FILL_ENOCONV) if allow_noconv else (FILL_OK,)
    return _check(_lib.fill_realize(plan, d_obs_ptr, C.c_uint64(seed), x_out_ptr, float(rtol)), "fill_realize", ok)


def fill_mean(plan, d_obs_ptr, x_out_ptr, rtol, allow_noconv=False):
    ok = (FILL_OK, FILL_ENOCONV) if allow_noconv else (FILL_OK,)
    return _check(_lib.fill_mean(plan, d_obs_ptr, x_out_ptr, float(rtol)), "fill_mean", ok)


def fill_get_stats(plan) -> dict:
    s = fill_stats()
    _check(_lib.fill_get_stats(plan, C.byref(s)), "fill_get_stats")
    return {k: getattr(s, k) for k, _ in fill_stats._fields_}


def fill_apply(plan, op, prec, in_ptr, out_ptr):
    return _check(_lib.fill_apply(plan, op, prec, in_ptr, out_ptr), "fill_apply")


def fill_realize_unconstrained(plan, seed, out_ptr):
    return _check(_lib.fill_realize_unconstrained(plan, C.c_uint64(seed), out_ptr), "fill_realize_unconstrained")


def fill_realize_unconstrained_noalloc(plan, seed, out_ptr):
    return _check(_lib.fill_realize_unconstrained_noalloc(plan, C.c_uint64(seed), out_ptr),
                  "fill_realize_unconstrained_noalloc")


def fill_philox_words(seed, stream, n_blocks, out_ptr):
    return _check(_lib.fill_philox_words(C.c_uint64(seed), C.c_uint64(stream), int(n_blocks), out_ptr),
                  "fill_philox_words")


def fill_time_kernel(plan, kernel, prec, reps) -> float:
    ms = C.c_double()
    _check(_lib.fill_time_kernel(plan, kernel, prec, int(reps), C.byref(ms)), "fill_time_kernel")
    return ms.value


def fill_kernel_timing(plan, kernel, prec):
    return _check(_lib.fill_kernel_timing(plan, int(kernel), int(prec)), "fill_kernel_timing")


def fill_kernel_timing_read(plan):
    ms, n = C.c_double(), C.c_int64()
    _check(_lib.fill_kernel_timing_read(plan, C.byref(ms), C.byref(n)), "fill_kernel_timing_read")
    return ms.value, n.value


def fill_strerror(code: int) -> str:
    return _strerror(code)


def fill_last_error() -> str:
    return _lib.fill_last_error().decode()


# ---- torch convenience -----------------------------------------------------

def _dev_ptr(t, dtype=None):
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


class Plan:
    """Owner of a fill_plan bound to a torch device stream."""

    def __init__(self, nx, ny, mask, Pk, prec=FILL_PREC_FP64, stream=None, device=None):
        import torch
        self.device = torch.device(device or "cuda")
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = s
            if hasattr(mask, "cpu"):
                mask = mask.cpu().numpy()
            if hasattr(Pk, "cpu"):
                Pk = Pk.cpu().numpy()
            self.nx, self.ny, self.prec = nx, ny, prec
            self.handle = fill_plan_create(nx, ny, mask, Pk, prec, s.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            fill_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_pk(self, Pk):
        if hasattr(Pk, "cpu"):
            Pk = Pk.cpu().numpy()
        fill_plan_set_pk(self.handle, Pk)

    def set_max_iter(self, n):
        fill_plan_set_max_iter(self.handle, n)

    def set_inner_tol(self, tol):
        fill_plan_set_inner_tol(self.handle, tol)

    def set_precond(self, mode):
        """Inner-CG preconditioner: FILL_PRECOND_SPLIT (default, or True), _CXX, _BLOCK or _NONE (False)."""
        fill_plan_set_precond(self.handle, mode)

    def set_cg(self, variant):
        """Inner-CG recurrence: FILL_CG_STANDARD (default) or FILL_CG_SINGLE_REDUCTION."""
        fill_plan_set_cg(self.handle, variant)

    def set_block_halo(self, halo):
        """Halo of the block preconditioner's pieces: 0..14 or FILL_BLOCK_HALO_AUTO (default)."""
        fill_plan_set_block_halo(self.handle, halo)

    def block_info(self) -> dict:
        """Size of the block preconditioner (FILL_PRECOND_BLOCK must be selected)."""
        return fill_get_block_info(self.handle)

    def set_graph(self, on):
        """Replay the inner-CG chunks as a captured HIP graph (default) or launch kernels one by one."""
        fill_plan_set_graph(self.handle, on)

    def laplace(self, d_obs, nkernels=8, r0=1.5, ratio=2.0, iters=100, out=None):
        """Kernel-based Laplace relaxation of the masked pixels (an approximate fill)."""
        import torch
        out = self._new_map() if out is None else out
        _check(_lib.fill_laplace(self.handle, _dev_ptr(d_obs, torch.float64), _dev_ptr(out, torch.float64),
                                 int(nkernels), float(r0), float(ratio), int(iters)), "fill_laplace")
        return out

    def set_skew(self, eps):
        """Non-Hermitian study: inner-CG A applies use Px C^-1 (I + eps K) Px (0 restores A)."""
        fill_plan_set_skew(self.handle, eps)

    def set_warm_start(self, iters, nkernels=8, r0=1.5, ratio=2.0):
        """Start later solves from the Laplace relaxation of the data (iters sweeps; 0 = off)."""
        fill_plan_set_warm_start(self.handle, iters, nkernels, r0, ratio)

    def set_lanczos(self, cap):
        """Record up to cap CG coefficients of the first inner solve of later solves."""
        fill_plan_set_lanczos(self.handle, cap)
        self.lanczos_cap = int(cap)

    def lanczos(self, problem=0):
        """(alpha, beta) recorded by the last solve."""
        return fill_get_lanczos(self.handle, problem, getattr(self, "lanczos_cap", 0))

    def lanczos_extremes(self, problem=0):
        """(lambda_min, lambda_max, steps): extreme Ritz values of the recorded Lanczos matrix."""
        return fill_lanczos_extremes(self.handle, problem)

    def _new_map(self):
        import torch
        return torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)

    def realize(self, d_obs, seed, rtol, out=None, allow_noconv=False):
        import torch
        out = self._new_map() if out is None else out
        fill_realize(self.handle, _dev_ptr(d_obs, torch.float64), seed, _dev_ptr(out, torch.float64), rtol,
                     allow_noconv)
        return out

    def mean(self, d_obs, rtol, out=None, allow_noconv=False):
        import torch
        out = self._new_map() if out is None else out
        fill_mean(self.handle, _dev_ptr(d_obs, torch.float64), _dev_ptr(out, torch.float64), rtol, allow_noconv)
        return out

    def apply(self, op, x, prec=None, out=None):
        import torch
        out = self._new_map() if out is None else out
        fill_apply(self.handle, op, self.prec if prec is None else prec, _dev_ptr(x, torch.float64),
                   _dev_ptr(out, torch.float64))
        return out

    def realize_unconstrained(self, seed, out=None):
        import torch
        out = self._new_map() if out is None else out
        fill_realize_unconstrained(self.handle, seed, _dev_ptr(out, torch.float64))
        return out

    def stats(self) -> dict:
        return fill_get_stats(self.handle)

    def set_bands(self, lnk_nodes, theta):
        fill_plan_set_bands(self.handle, lnk_nodes, theta)
        self.nbands = len(lnk_nodes)

    def adjoint(self, d_obs, seed, x_out, g, rtol=1e-10, want_logP=False, allow_noconv=False):
        """(grad_dobs, grad_theta, grad_logP) of a loss with dL/dx_out = g."""
        import torch
        grad_d = torch.empty_like(d_obs)
        for t in (d_obs, x_out, g, grad_d):
            _dev_ptr(t, torch.float64)
        gth, glp = fill_adjoint_batch(self.handle, [d_obs.data_ptr()], [seed], [x_out.data_ptr()], [g.data_ptr()],
                                      [grad_d.data_ptr()], getattr(self, "nbands", 0),
                                      nt=self.ny * (self.nx // 2 + 1), rtol=rtol, want_logP=want_logP,
                                      allow_noconv=allow_noconv)
        if glp is not None:
            glp = glp.reshape(self.ny, self.nx // 2 + 1)
        return grad_d, gth, glp

    def kernel_timing(self, kernel, prec=None):
        """Time every launch of `kernel` during later solves with HIP events (-1 = off)."""
        fill_kernel_timing(self.handle, kernel, self.prec if prec is None else prec)

    def kernel_timing_read(self):
        """(total ms, launches) since the last read; synchronises the plan's stream."""
        return fill_kernel_timing_read(self.handle)

    def time_kernel(self, kernel, reps=50, prec=None) -> float:
        """Average milliseconds per launch of one kernel of the A apply."""
        return fill_time_kernel(self.handle, kernel, self.prec if prec is None else prec, reps)


class BatchPlan:
    """Owner of a batched fill_plan (nprob same-size problems) on a torch stream."""

    def __init__(self, nx, ny, masks, Pk, prec=FILL_PREC_FP64, stream=None, device=None):
        import torch
        self.device = torch.device(device or "cuda")
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = s
            if hasattr(masks, "cpu"):
                masks = masks.cpu().numpy()
            if hasattr(Pk, "cpu"):
                Pk = Pk.cpu().numpy()
            self.nx, self.ny, self.prec = nx, ny, prec
            self.handle = fill_plan_create_batch(nx, ny, masks, Pk, prec, s.cuda_stream)
            self.nprob = fill_plan_nprob(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            fill_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def realize(self, d_obs, seeds, rtol, out=None, allow_noconv=False):
        """d_obs: device float64 (nprob, ny, nx); returns x_out of the same shape."""
        import torch
        out = torch.empty_like(d_obs) if out is None else out
        if d_obs.shape != (self.nprob, self.ny, self.nx) or out.shape != d_obs.shape:
            raise ValueError("d_obs/out must be (nprob, ny, nx)")
        _dev_ptr(d_obs, torch.float64)
        _dev_ptr(out, torch.float64)
        fill_realize_batch(self.handle, [d_obs[b].data_ptr() for b in range(self.nprob)], seeds,
                           [out[b].data_ptr() for b in range(self.nprob)], rtol, allow_noconv)
        return out

    def mean(self, d_obs, rtol, out=None, allow_noconv=False):
        import torch
        out = torch.empty_like(d_obs) if out is None else out
        _dev_ptr(d_obs, torch.float64)
        _dev_ptr(out, torch.float64)
        fill_mean_batch(self.handle, [d_obs[b].data_ptr() for b in range(self.nprob)],
                        [out[b].data_ptr() for b in range(self.nprob)], rtol, allow_noconv)
        return out

    def stats(self) -> list:
        return fill_get_stats_batch(self.handle)

    def kernel_timing(self, kernel, prec=None):
        fill_kernel_timing(self.handle, kernel, self.prec if prec is None else prec)

    def kernel_timing_read(self):
        return fill_kernel_timing_read(self.handle)

    def set_inner_tol(self, tol):
        fill_plan_set_inner_tol(self.handle, tol)

    def set_max_iter(self, n):
        fill_plan_set_max_iter(self.handle, n)

    def set_bands(self, lnk_nodes, theta):
        fill_plan_set_bands(self.handle, lnk_nodes, theta)
        self.nbands = len(lnk_nodes)

    def set_precond(self, mode):
        """Inner-CG preconditioner: FILL_PRECOND_SPLIT (default, or True), _CXX, _BLOCK or _NONE (False)."""
        fill_plan_set_precond(self.handle, mode)

    def set_cg(self, variant):
        """Inner-CG recurrence: FILL_CG_STANDARD (default) or FILL_CG_SINGLE_REDUCTION."""
        fill_plan_set_cg(self.handle, variant)

    def set_block_halo(self, halo):
        """Halo of the block preconditioner's pieces: 0..14 or FILL_BLOCK_HALO_AUTO (default)."""
        fill_plan_set_block_halo(self.handle, halo)

    def block_info(self) -> dict:
        """Size of the block preconditioner (FILL_PRECOND_BLOCK must be selected)."""
        return fill_get_block_info(self.handle)

    def set_graph(self, on):
        """Replay the inner-CG chunks as a captured HIP graph (default) or launch kernels one by one."""
        fill_plan_set_graph(self.handle, on)

    def laplace(self, d_obs, nkernels=8, r0=1.5, ratio=2.0, iters=100, out=None):
        """Kernel-based Laplace relaxation of the masked pixels (an approximate fill)."""
        import torch
        out = self._new_map() if out is None else out
        _check(_lib.fill_laplace(self.handle, _dev_ptr(d_obs, torch.float64), _dev_ptr(out, torch.float64),
                                 int(nkernels), float(r0), float(ratio), int(iters)), "fill_laplace")
        return out

    def set_skew(self, eps):
        """Non-Hermitian study: inner-CG A applies use Px C^-1 (I + eps K) Px (0 restores A)."""
        fill_plan_set_skew(self.handle, eps)

    def set_warm_start(self, iters, nkernels=8, r0=1.5, ratio=2.0):
        """Start later solves from the Laplace relaxation of the data (iters sweeps; 0 = off)."""
        fill_plan_set_warm_start(self.handle, iters, nkernels, r0, ratio)

    def set_lanczos(self, cap):
        """Record up to cap CG coefficients of the first inner solve of later solves."""
        fill_plan_set_lanczos(self.handle, cap)
        self.lanczos_cap = int(cap)

    def lanczos(self, problem=0):
        """(alpha, beta) recorded by the last solve."""
        return fill_get_lanczos(self.handle, problem, getattr(self, "lanczos_cap", 0))

    def lanczos_extremes(self, problem=0):
        """(lambda_min, lambda_max, steps): extreme Ritz values of the recorded Lanczos matrix."""
        return fill_lanczos_extremes(self.handle, problem)

    def adjoint(self, d_obs, seeds, x_out, g, rtol=1e-10, want_logP=False, allow_noconv=False):
        """(grad_dobs, grad_theta, grad_logP) of a loss with dL/dx_out = g (all (nprob, ny, nx))."""
        import torch
        grad_d = torch.empty_like(d_obs)
        for t in (d_obs, x_out, g, grad_d):
            _dev_ptr(t, torch.float64)
        n = self.nprob
        gth, glp = fill_adjoint_batch(self.handle, [d_obs[b].data_ptr() for b in range(n)], seeds,
                                      [x_out[b].data_ptr() for b in range(n)], [g[b].data_ptr() for b in range(n)],
                                      [grad_d[b].data_ptr() for b in range(n)], getattr(self, "nbands", 0),
                                      nt=self.ny * (self.nx // 2 + 1), rtol=rtol, want_logP=want_logP,
                                      allow_noconv=allow_noconv)
        if glp is not None:
            glp = glp.reshape(n, self.ny, self.nx // 2 + 1)
        return grad_d, gth, glp


def realize_multi(plans, d_obs_list, seeds_list, rtol, outs=None, allow_noconv=False):
    """Run several BatchPlans concurrently (one host thread each)."""
    import torch
    outs = outs if outs is not None else [torch.empty_like(d) for d in d_obs_list]
    fill_realize_multi([p.handle for p in plans],
                       [[d[b].data_ptr() for b in range(p.nprob)] for p, d in zip(plans, d_obs_list)],
                       seeds_list,
                       [[o[b].data_ptr() for b in range(p.nprob)] for p, o in zip(plans, outs)],
                       rtol, allow_noconv)
    return outs


class Group:
    """Several BatchPlans (for example one per grid size) solved together:
    after a first step-by-step call, every call is one graph launch on the
    group's stream (see fill_group_realize)."""

    def __init__(self, plans, stream=None):
        import torch
        self.plans = list(plans)
        dev = self.plans[0].device
        with torch.cuda.device(dev):
            s = stream if stream is not None else torch.cuda.current_stream(dev)
        self.stream = s
        self.handle = fill_group_create([p.handle for p in self.plans], s.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            fill_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def realize(self, d_obs_list, seeds_list, rtol, outs=None, allow_noconv=False):
        import torch
        outs = outs if outs is not None else [torch.empty_like(d) for d in d_obs_list]
        for d, o in zip(d_obs_list, outs):
            _dev_ptr(d, torch.float64)
            _dev_ptr(o, torch.float64)
        fill_group_realize(self.handle,
                           [[d[b].data_ptr() for b in range(p.nprob)] for p, d in zip(self.plans, d_obs_list)],
                           seeds_list,
                           [[o[b].data_ptr() for b in range(p.nprob)] for p, o in zip(self.plans, outs)],
                           rtol, allow_noconv)
        return outs

    def last_graph(self) -> bool:
        return fill_group_last_graph(self.handle)


def _check_strips(code: int, where: str, ok=(FILL_OK,)) -> int:
    if code not in ok:
        raise FillError(code, where, _lib.fill_strips_last_error().decode())
    return code


class Strips:
    """Owner of a fill_strips object (noise-boosted strip refinement) on a torch stream."""

    def __init__(self, nx, ny, mask, P_signal, noise, betas, widths, threshold=0.03, iters=20,
                 prec=FILL_PREC_FP64, stream=None, device=None):
        import torch
        self.device = torch.device(device or "cuda")
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            P = np.ascontiguousarray(P_signal, dtype=np.float64)
            if m.shape != (ny, nx) or P.shape != (ny, nx // 2 + 1):
                raise ValueError("mask / P_signal do not match the grid")
            b = np.ascontiguousarray(betas, dtype=np.float64)
            w = np.ascontiguousarray(widths, dtype=np.float64)
            if b.shape != w.shape or b.ndim != 1:
                raise ValueError("betas and widths must be 1-D of equal length")
            h = C.c_void_p()
            _check_strips(_lib.fill_strips_create(nx, ny, m.ctypes.data, P.ctypes.data, float(noise), len(b),
                                                  b.ctypes.data, w.ctypes.data, float(threshold), int(iters),
                                                  int(prec), C.c_void_p(s.cuda_stream), C.byref(h)),
                          "fill_strips_create")
            self.handle, self.nx, self.ny, self.nstrips = h.value, nx, ny, len(b)

    def close(self):
        if getattr(self, "handle", None):
            _lib.fill_strips_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mean(self, d_obs, out=None):
        import torch
        out = torch.empty_like(d_obs) if out is None else out
        _check_strips(_lib.fill_strips_mean(self.handle, _dev_ptr(d_obs, torch.float64),
                                            _dev_ptr(out, torch.float64)), "fill_strips_mean")
        return out

    def refine(self, x):
        """The strip sequence on a filled map (data on observed pixels, a start on masked ones), in place."""
        import torch
        _check_strips(_lib.fill_strips_refine(self.handle, _dev_ptr(x, torch.float64)), "fill_strips_refine")
        return x

    def mask(self, i):
        out = np.zeros((self.ny, self.nx), np.uint8)
        _check_strips(_lib.fill_strips_mask(self.handle, int(i), out.ctypes.data), "fill_strips_mask")
        return out

    def plan(self, i):
        """The raw fill_plan handle of strip i (None for an empty strip); owned by this object."""
        h = C.c_void_p()
        _check_strips(_lib.fill_strips_plan(self.handle, int(i), C.byref(h)), "fill_strips_plan")
        return h.value


def philox_words(seed, stream, n_blocks, device="cuda"):
    import torch
    out = torch.empty(4 * n_blocks, dtype=torch.int64, device=device)
    fill_philox_words(seed, stream, n_blocks, out.data_ptr())
    return out
