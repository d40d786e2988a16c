"""Python binding of libadkion (ctypes over the C ABI in include/adkion.h).

Argument marshalling only: every step of the ionization path runs in the HIP
kernels of libadkion.so.  Device arrays are torch tensors on a ROCm device
(torch is used for device memory and streams).  If the library is not built
the first call raises; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadkion.so")

ADK_OK, ADK_EINVAL, ADK_ERANGE, ADK_EDEVICE, ADK_ENOMEM = 0, -1, -2, -3, -4
ADK_F64, ADK_MIXED = 0, 1
ADK_LAYOUT_COMPACT, ADK_LAYOUT_FULL = 0, 1
ADK_MAX_Z, ADK_MAX_W, ADK_MAX_WIDE_W, ADK_M_AVERAGE = 64, 8, 63, -1
ADK_MLP_NOALLOC_MAX_SAMPLES = 4096

#: every function the header declares (checked by the CPU test suite)
EXPORTS = ("adk_version", "adk_strerror", "adk_gas_coeffs", "adk_gas_create", "adk_gas_destroy",
           "adk_gas_levels", "adk_rates", "adk_chain_advance", "ionize_step", "ionize_step_yield",
           "adk_subcycle_step", "adk_plan_create",
           "adk_plan_step", "adk_plan_graph_replay", "adk_plan_get_info", "adk_plan_order", "adk_plan_destroy", "adk_field_hash", "adk_mlp_nparams",
           "adk_mlp_create", "adk_mlp_destroy", "adk_mlp_get_state", "adk_band_columns", "adk_mlp_forward",
           "adk_mlp_loss_grad", "adk_mlp_train", "adk_mlp_save", "adk_mlp_load", "adk_surrogate_step",
           "adk_ceiling_copy", "adk_ceiling_valu", "adk_adaptive_work_bytes", "ionize_step_adaptive",
           "adk_mlp_loss_grad_noalloc", "adk_mlp_forward_trace")
ADK_PLAN_MAX_GAS, ADK_PLAN_MAX_W = 8, 6


class AdkError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_text(status)} ({status})")


class _Consts(ctypes.Structure):
    _fields_ = [("omega_a", ctypes.c_double), ("E_a", ctypes.c_double), ("U_H", ctypes.c_double)]


class _GasDesc(ctypes.Structure):
    _fields_ = [("Z", ctypes.c_int32), ("U_eV", ctypes.POINTER(ctypes.c_double)),
                ("l", ctypes.POINTER(ctypes.c_int8)), ("m", ctypes.POINTER(ctypes.c_int8))]


PLAN_MAX_W = 6
ADK_PLAN_MESH_ORDER, ADK_PLAN_GROUPED = 0, 1


class _PlanInfo(ctypes.Structure):
    _fields_ = [("ngas", ctypes.c_int32), ("nbuckets", ctypes.c_int32), ("ntiles", ctypes.c_int32),
                ("cells_per_lane", ctypes.c_int32), ("grid", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("from_cache", ctypes.c_int32), ("tuned_us", ctypes.c_double), ("nlaunches", ctypes.c_int32),
                ("launch_wmax", ctypes.c_int32 * PLAN_MAX_W), ("launch_cpl", ctypes.c_int32 * PLAN_MAX_W),
                ("launch_grid", ctypes.c_int32 * PLAN_MAX_W), ("launch_tiles", ctypes.c_int32 * PLAN_MAX_W),
                ("launch_cells", ctypes.c_int64 * PLAN_MAX_W), ("layout", ctypes.c_int32)]


class _MlpRange(ctypes.Structure):
    _fields_ = [("E_lo", ctypes.c_double), ("E_hi", ctypes.c_double), ("dt_lo", ctypes.c_double),
                ("dt_hi", ctypes.c_double)]


class _TrainCfg(ctypes.Structure):
    _fields_ = [("nsamples", ctypes.c_int64), ("iters", ctypes.c_int32), ("total_iters", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_double), ("lr_min", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class _Window(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("eps", ctypes.c_double), ("layout", ctypes.c_int),
                ("prec", ctypes.c_int)]


class _Adaptive(ctypes.Structure):
    _fields_ = [("wmin", ctypes.c_int32), ("wmax", ctypes.c_int32), ("eps", ctypes.c_double),
                ("tol", ctypes.c_double), ("prec", ctypes.c_int)]


_lib = None


def _sig(L, name, attr, value):
    """Set a symbol's ctypes signature; a symbol the loaded library lacks is
    left for the call itself to report (the CPU tests check that the built
    library exports every declared function)."""
    if hasattr(L, name):
        setattr(getattr(L, name), attr, value)


def lib():
    """Load libadkion.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2202_10647_amd.build` "
                           "(no fallback path exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    _sig(L, "adk_version", "restype", ctypes.c_char_p)
    _sig(L, "adk_version", "argtypes", [])
    _sig(L, "adk_strerror", "restype", ctypes.c_char_p)
    _sig(L, "adk_strerror", "argtypes", [ctypes.c_int])
    _sig(L, "adk_gas_coeffs", "restype", ctypes.c_int)
    _sig(L, "adk_gas_coeffs", "argtypes", [ctypes.POINTER(_GasDesc), ctypes.POINTER(_Consts), ctypes.POINTER(dbl)])
    _sig(L, "adk_gas_create", "restype", ctypes.c_int)
    _sig(L, "adk_gas_create", "argtypes", [ctypes.POINTER(_GasDesc), ctypes.POINTER(_Consts), ctypes.POINTER(vp)])
    _sig(L, "adk_gas_destroy", "restype", ctypes.c_int)
    _sig(L, "adk_gas_destroy", "argtypes", [vp])
    _sig(L, "adk_gas_levels", "restype", ctypes.c_int)
    _sig(L, "adk_gas_levels", "argtypes", [vp])
    _sig(L, "adk_rates", "restype", ctypes.c_int)
    _sig(L, "adk_rates", "argtypes", [vp, vp, i64, i32, i32, vp, ctypes.c_int, vp])
    _sig(L, "adk_chain_advance", "restype", ctypes.c_int)
    _sig(L, "adk_chain_advance", "argtypes", [i32, vp, i64, dbl, vp, ctypes.c_int, vp])
    _sig(L, "ionize_step", "restype", ctypes.c_int)
    _sig(L, "ionize_step", "argtypes", [vp, vp, i64, dbl, vp, vp, ctypes.POINTER(_Window), vp])
    _sig(L, "adk_adaptive_work_bytes", "restype", ctypes.c_size_t)
    _sig(L, "adk_adaptive_work_bytes", "argtypes", [i64])
    _sig(L, "ionize_step_adaptive", "restype", ctypes.c_int)
    _sig(L, "ionize_step_adaptive", "argtypes", [vp, vp, i64, dbl, vp, vp, vp, ctypes.POINTER(_Adaptive), vp,
                                                 ctypes.c_size_t, vp, vp])
    _sig(L, "adk_subcycle_step", "restype", ctypes.c_int)
    _sig(L, "adk_subcycle_step", "argtypes", [vp, vp, i64, dbl, vp, vp, ctypes.POINTER(_Window), i32, vp])
    _sig(L, "ionize_step_yield", "restype", ctypes.c_int)
    _sig(L, "ionize_step_yield", "argtypes", [vp, vp, i64, dbl, vp, vp, ctypes.POINTER(_Window), vp, vp])
    _sig(L, "adk_plan_create", "restype", ctypes.c_int)
    _sig(L, "adk_plan_create", "argtypes", [ctypes.POINTER(vp), i32, vp, vp, i64, ctypes.c_int, dbl, i32, i32,
                                            ctypes.POINTER(vp)])
    _sig(L, "adk_plan_order", "restype", ctypes.c_int)
    _sig(L, "adk_plan_order", "argtypes", [vp, vp])
    _sig(L, "adk_plan_step", "restype", ctypes.c_int)
    _sig(L, "adk_plan_step", "argtypes", [vp, vp, dbl, vp, vp, vp])
    _sig(L, "adk_plan_graph_replay", "restype", ctypes.c_int)
    _sig(L, "adk_plan_graph_replay", "argtypes", [vp, i32, vp])
    _sig(L, "adk_plan_get_info", "restype", ctypes.c_int)
    _sig(L, "adk_plan_get_info", "argtypes", [vp, ctypes.POINTER(_PlanInfo)])
    _sig(L, "adk_plan_destroy", "restype", ctypes.c_int)
    _sig(L, "adk_plan_destroy", "argtypes", [vp])
    _sig(L, "adk_field_hash", "restype", ctypes.c_int)
    _sig(L, "adk_field_hash", "argtypes", [vp, i64, ctypes.c_uint64, i64, dbl, dbl, ctypes.c_int, vp])
    _sig(L, "adk_ceiling_copy", "restype", ctypes.c_int)
    _sig(L, "adk_ceiling_copy", "argtypes", [vp, vp, i64, i64, vp])
    _sig(L, "adk_ceiling_valu", "restype", ctypes.c_int)
    _sig(L, "adk_ceiling_valu", "argtypes", [i32, i64, vp, i64, vp])
    _sig(L, "adk_mlp_nparams", "restype", i64)
    _sig(L, "adk_mlp_nparams", "argtypes", [i32])
    _sig(L, "adk_mlp_create", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_create", "argtypes", [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_MlpRange), ctypes.POINTER(vp)])
    _sig(L, "adk_mlp_destroy", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_destroy", "argtypes", [vp])
    _sig(L, "adk_mlp_get_state", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_get_state", "argtypes", [vp, vp, vp, vp, ctypes.POINTER(i64)])
    _sig(L, "adk_band_columns", "restype", ctypes.c_int)
    _sig(L, "adk_band_columns", "argtypes", [vp, vp, vp, vp, i64, vp, vp])
    _sig(L, "adk_mlp_forward", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_forward", "argtypes", [vp, vp, vp, vp, i64, vp, vp])
    _sig(L, "adk_mlp_loss_grad", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_loss_grad", "argtypes", [vp, vp, vp, vp, vp, i64, vp, vp, vp])
    _sig(L, "adk_mlp_forward_trace", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_forward_trace", "argtypes", [vp, vp, vp, vp, i64, vp, vp, vp])
    _sig(L, "adk_mlp_loss_grad_noalloc", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_loss_grad_noalloc", "argtypes", [vp, vp, vp, vp, vp, i64, vp, vp, vp])
    _sig(L, "adk_mlp_train", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_train", "argtypes", [vp, vp, ctypes.POINTER(_TrainCfg), vp, vp])
    _sig(L, "adk_mlp_save", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_save", "argtypes", [vp, ctypes.c_char_p])
    _sig(L, "adk_mlp_load", "restype", ctypes.c_int)
    _sig(L, "adk_mlp_load", "argtypes", [vp, ctypes.c_char_p, ctypes.POINTER(vp)])
    _sig(L, "adk_surrogate_step", "restype", ctypes.c_int)
    _sig(L, "adk_surrogate_step", "argtypes", [vp, vp, vp, i64, dbl, vp, vp, ctypes.POINTER(_Window), vp, vp])
    _lib = L
    return L


def status_text(status: int) -> str:
    try:
        return lib().adk_strerror(int(status)).decode()
    except RuntimeError:
        return "library not built"


def version() -> str:
    return lib().adk_version().decode()


def _check(st: int, what: str):
    if st != ADK_OK:
        raise AdkError(st, what)


def _desc(U, l, m):
    U = np.ascontiguousarray(np.asarray(U, dtype=np.float64))
    l = np.ascontiguousarray(np.asarray(l, dtype=np.int8))
    m = np.ascontiguousarray(np.asarray(m, dtype=np.int8))
    d = _GasDesc(int(U.size), U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 l.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                 m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return d, (U, l, m)


def _consts(consts):
    if consts is None:
        return None
    return ctypes.pointer(_Consts(*[float(c) for c in consts]))


def gas_coeffs(U, l, m, consts=None) -> np.ndarray:
    """Host-only log-domain coefficient table [Z][8] (A, alpha, B, c1, c2, c3, 0, 0)."""
    d, keep = _desc(U, l, m)
    out = np.zeros((max(d.Z, 1), 8), dtype=np.float64)
    st = lib().adk_gas_coeffs(ctypes.byref(d), _consts(consts),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(st, "adk_gas_coeffs")
    return out[: d.Z]


class Gas:
    """A gas level table uploaded to the current device (owned by the library)."""

    def __init__(self, U, l, m, consts=None):
        d, keep = _desc(U, l, m)
        h = ctypes.c_void_p()
        st = lib().adk_gas_create(ctypes.byref(d), _consts(consts), ctypes.byref(h))
        _check(st, "adk_gas_create")
        self._h = h
        self.Z = int(d.Z)

    @classmethod
    def from_table(cls, table, consts=None):
        return cls(table.U, table.l, table.m, consts)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().adk_gas_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _prec_of(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return ADK_F64
    if t.dtype == torch.float32:
        return ADK_MIXED
    raise TypeError(f"unsupported dtype {t.dtype}: float64 (ADK_F64) or float32 (ADK_MIXED)")


def _dev(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def rates(gas: Gas, E, k0: int = 0, nk: Optional[int] = None, out=None, stream=None):
    """W[nk][n] (1/s) of levels k0..k0+nk-1 at fields E[n] (float64 or float32)."""
    import torch
    if nk is None:
        nk = gas.Z - k0
    n = E.numel()
    if out is None:
        out = torch.empty((nk, n), dtype=E.dtype, device=E.device)
    st = lib().adk_rates(gas.handle, _dev(E, "E"), n, k0, nk, _dev(out, "W_out"), _prec_of(E),
                         _stream(stream))
    _check(st, "adk_rates")
    return out


def chain_advance(W, dt: float, pops, stream=None):
    """In place: pops[(w+1)][n] <- expm(dt A(W)) pops with rates W[w][n] (1/s)."""
    w = W.shape[0]
    n = pops.shape[1] if pops.dim() == 2 else 0
    if pops.dtype != W.dtype or pops.shape[0] != w + 1 or W.shape[1] != n:
        raise ValueError("W must be [w][n] and pops [(w+1)][n] of the same dtype")
    st = lib().adk_chain_advance(w, _dev(W, "W"), n, float(dt), _dev(pops, "pops"), _prec_of(pops),
                                 _stream(stream))
    _check(st, "adk_chain_advance")
    return pops


def ionize_step(gas: Gas, E, dt: float, pops, lo, w: int, eps: float = 1e-8, layout: str = "compact",
                stream=None, dne=None):
    """One ionization step, in place on pops and lo (see include/adkion.h).

    float64 tensors select ADK_F64, float32 tensors ADK_MIXED.  With dne (a
    device tensor of E's dtype and size, compact layout) the step also writes
    each cell's electron yield (ionize_step_yield)."""
    import torch
    lay = {"compact": ADK_LAYOUT_COMPACT, "full": ADK_LAYOUT_FULL}[layout]
    n = E.numel()
    rows = (w + 1) if lay == ADK_LAYOUT_COMPACT else (gas.Z + 1)
    if pops.dtype != E.dtype or tuple(pops.shape) != (rows, n):
        raise ValueError(f"pops must be [{rows}][{n}] of dtype {E.dtype}, got {tuple(pops.shape)} {pops.dtype}")
    if lo.dtype != torch.uint8 or lo.numel() != n:
        raise ValueError("lo must be uint8[ncells]")
    win = _Window(int(w), float(eps), lay, _prec_of(E))
    if dne is not None:
        if dne.dtype != E.dtype or dne.numel() != n:
            raise ValueError("dne must match E in dtype and size")
        st = lib().ionize_step_yield(gas.handle, _dev(E, "E"), n, float(dt), _dev(pops, "pops"), _dev(lo, "lo"),
                                     ctypes.byref(win), _dev(dne, "dne"), _stream(stream))
        _check(st, "ionize_step_yield")
        return pops, lo
    st = lib().ionize_step(gas.handle, _dev(E, "E"), n, float(dt), _dev(pops, "pops"), _dev(lo, "lo"),
                           ctypes.byref(win), _stream(stream))
    _check(st, "ionize_step")
    return pops, lo


def adaptive_work_bytes(ncells: int) -> int:
    """Bytes of the device workspace ionize_step_adaptive needs for ncells cells."""
    return int(lib().adk_adaptive_work_bytes(int(ncells)))


def adaptive_workspace(ncells: int, device="cuda"):
    """A device workspace for ionize_step_adaptive (a uint8 tensor)."""
    import torch
    return torch.empty(adaptive_work_bytes(ncells), dtype=torch.uint8, device=device)


def ionize_step_adaptive(gas: Gas, E, dt: float, pops, lo, wc, wmin: int, wmax: int, eps: float = 1e-8,
                         tol: float = 1e-9, work=None, counters=None, stream=None):
    """One step with per-cell adaptive windows, in place on pops
    [(wmax+1)][ncells], lo and wc (uint8[ncells]); see include/adkion.h.
    float64 tensors select ADK_F64, float32 tensors ADK_MIXED.  work: a
    device workspace (adaptive_workspace); counters: optional int64[2]."""
    import torch
    n = E.numel()
    if pops.dtype != E.dtype or tuple(pops.shape) != (wmax + 1, n):
        raise ValueError(f"pops must be [{wmax + 1}][{n}] of dtype {E.dtype}, got {tuple(pops.shape)} {pops.dtype}")
    for t, name in ((lo, "lo"), (wc, "wc")):
        if t.dtype != torch.uint8 or t.numel() != n:
            raise ValueError(f"{name} must be uint8[ncells]")
    if work is None:
        raise ValueError("work: a device workspace of adaptive_work_bytes(ncells) bytes is required")
    if counters is not None and (counters.dtype != torch.int64 or counters.numel() < 2):
        raise ValueError("counters must be int64[2]")
    win = _Adaptive(int(wmin), int(wmax), float(eps), float(tol), _prec_of(E))
    st = lib().ionize_step_adaptive(gas.handle, _dev(E, "E"), n, float(dt), _dev(pops, "pops"), _dev(lo, "lo"),
                                    _dev(wc, "wc"), ctypes.byref(win), _dev(work, "work"),
                                    work.numel() * work.element_size(),
                                    _dev(counters, "counters") if counters is not None else None, _stream(stream))
    _check(st, "ionize_step_adaptive")
    return pops, lo, wc


def subcycle_step(gas: Gas, E, dt: float, pops, lo, w: int, nsub: int, eps: float = 1e-8, stream=None):
    """Comparison baseline: the step with nsub explicit RK4 substeps instead of
    the analytic chain solution (float64 tensors, compact layout), in place."""
    import torch
    n = E.numel()
    if E.dtype != torch.float64 or pops.dtype != torch.float64 or tuple(pops.shape) != (w + 1, n):
        raise ValueError(f"E float64[{n}] and pops float64[{w + 1}][{n}] expected")
    if lo.dtype != torch.uint8 or lo.numel() != n:
        raise ValueError("lo must be uint8[ncells]")
    win = _Window(int(w), float(eps), ADK_LAYOUT_COMPACT, ADK_F64)
    st = lib().adk_subcycle_step(gas.handle, _dev(E, "E"), n, float(dt), _dev(pops, "pops"), _dev(lo, "lo"),
                                 ctypes.byref(win), int(nsub), _stream(stream))
    _check(st, "adk_subcycle_step")
    return pops, lo


class Plan:
    """Batched step over cells of several gases (see adk_plan_create).

    gases: list of Gas; cell_gas, cell_w: per-cell gas index and window width
    (host arrays, mesh order); prec: "mixed" (float) or "f64"; cells_per_lane:
    0 = autotune; layout: "mesh" (arrays indexed by mesh cell) or "grouped"
    (arrays in the plan's order, see order()).  Populations use
    pops[info.rows][ncells] (compact slots per cell)."""

    def __init__(self, gases, cell_gas, cell_w, prec="mixed", eps=1e-8, cells_per_lane=0, layout="mesh"):
        cg = np.ascontiguousarray(np.asarray(cell_gas, dtype=np.uint8))
        cw = np.ascontiguousarray(np.asarray(cell_w, dtype=np.uint8))
        if cg.shape != cw.shape or cg.ndim != 1:
            raise ValueError("cell_gas and cell_w must be 1-D arrays of one length")
        arr = (ctypes.c_void_p * max(1, len(gases)))(*[g.handle.value for g in gases])
        h = ctypes.c_void_p()
        self._prec = {"mixed": ADK_MIXED, "f64": ADK_F64}[prec]
        st = lib().adk_plan_create(arr, len(gases), cg.ctypes.data_as(ctypes.c_void_p),
                                   cw.ctypes.data_as(ctypes.c_void_p), int(cg.size), self._prec, float(eps),
                                   int(cells_per_lane),
                                   {"mesh": ADK_PLAN_MESH_ORDER, "grouped": ADK_PLAN_GROUPED}[layout],
                                   ctypes.byref(h))
        _check(st, "adk_plan_create")
        self._h = h
        self._gases = list(gases)  # keep the gas tables alive
        self.ncells = int(cg.size)
        self.info = self.get_info()

    def get_info(self) -> dict:
        inf = _PlanInfo()
        _check(lib().adk_plan_get_info(self._h, ctypes.byref(inf)), "adk_plan_get_info")
        out = {}
        for k, _ in _PlanInfo._fields_:
            v = getattr(inf, k)
            out[k] = list(v)[: inf.nlaunches] if k.startswith("launch_") else v
        return out

    def order(self):
        """adk_plan_order: int32[ncells], the mesh cell at each plan position."""
        out = np.empty(self.ncells, dtype=np.int32)
        _check(lib().adk_plan_order(self._h, out.ctypes.data_as(ctypes.c_void_p)), "adk_plan_order")
        return out

    def step(self, E, dt: float, pops, lo, stream=None):
        import torch
        want = torch.float32 if self._prec == ADK_MIXED else torch.float64
        if E.dtype != want or pops.dtype != want or E.numel() != self.ncells:
            raise ValueError("E/pops dtype or size does not match the plan")
        if tuple(pops.shape) != (self.info["rows"], self.ncells) or lo.dtype != torch.uint8:
            raise ValueError(f"pops must be [{self.info['rows']}][{self.ncells}], lo uint8[{self.ncells}]")
        st = lib().adk_plan_step(self._h, _dev(E, "E"), float(dt), _dev(pops, "pops"), _dev(lo, "lo"),
                                 _stream(stream))
        _check(st, "adk_plan_step")

    def graph_replay(self, nsteps: int, stream=None):
        """nsteps more steps with the arguments of the last step(), replayed
        as one captured hipGraph (captured on first use, cached)."""
        _check(lib().adk_plan_graph_replay(self._h, int(nsteps), _stream(stream)), "adk_plan_graph_replay")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().adk_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def field_hash(E, seed: int, step: int, E_lo: float = 10.0, E_hi: float = 5000.0, stream=None):
    """Fill the device tensor E with the seeded log-uniform synthetic field of
    (seed, step) (input generator; workloads.hash_field is its host twin)."""
    st = lib().adk_field_hash(_dev(E, "E"), E.numel(), int(seed) & 0xFFFFFFFFFFFFFFFF, int(step), float(E_lo),
                              float(E_hi), _prec_of(E), _stream(stream))
    _check(st, "adk_field_hash")
    return E


def ceiling_copy(dst, src, reps: int = 1, stream=None):
    """Measurement harness: reps passes of a streaming copy src -> dst (device
    tensors of equal byte size, a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise AdkError(ADK_EINVAL, "ceiling_copy: dst and src differ in size")
    _check(lib().adk_ceiling_copy(_dev(dst, "dst"), _dev(src, "src"), nbytes, int(reps), _stream(stream)),
           "adk_ceiling_copy")
    return dst


def ceiling_valu(kind: int, iters: int, out, stream=None):
    """Measurement harness: 8 dependency chains of `iters` float FMAs (kind 0),
    double FMAs (kind 1) or float exp2 (kind 2) per lane of out (one lane per
    element; float32 for kinds 0 and 2, float64 for kind 1)."""
    want = "float64" if kind == 1 else "float32"
    if str(out.dtype).split(".")[-1] != want:
        raise AdkError(ADK_EINVAL, f"ceiling_valu: kind {kind} writes {want}")
    _check(lib().adk_ceiling_valu(int(kind), int(iters), _dev(out, "out"), out.numel(), _stream(stream)),
           "adk_ceiling_valu")
    return out


# ---------------------------------------------------------------------------
# Band-column surrogate (see include/adkion.h)

def mlp_nparams(Z: int) -> int:
    return int(lib().adk_mlp_nparams(int(Z)))


def band_columns(gas: Gas, E, dt, k, out=None, stream=None):
    """Exact FP64 band columns cols[4][n] of samples (E, dt, k): float64 E and
    dt, int32 k device tensors."""
    import torch
    n = E.numel()
    if E.dtype != torch.float64 or dt.dtype != torch.float64 or k.dtype != torch.int32:
        raise ValueError("E, dt must be float64 and k int32")
    if dt.numel() != n or k.numel() != n:
        raise ValueError("E, dt, k must have one length")
    if out is None:
        out = torch.empty((4, n), dtype=torch.float64, device=E.device)
    st = lib().adk_band_columns(gas.handle, _dev(E, "E"), _dev(dt, "dt"), _dev(k, "k"), n, _dev(out, "cols"),
                                _stream(stream))
    _check(st, "adk_band_columns")
    return out


class Mlp:
    """The band-column network of one gas (weights, Adam state, training)."""

    def __init__(self, gas: Gas, params=None, E_range=(10.0, 5000.0), dt_range=(0.02e-15, 0.2e-15), _handle=None):
        self._gas = gas
        self.Z = gas.Z
        self.nparams = mlp_nparams(gas.Z)
        if _handle is not None:
            self._h = _handle
            return
        prm = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if prm.size != self.nparams:
            raise ValueError(f"params must have {self.nparams} entries")
        rng = _MlpRange(float(E_range[0]), float(E_range[1]), float(dt_range[0]), float(dt_range[1]))
        h = ctypes.c_void_p()
        st = lib().adk_mlp_create(gas.handle, prm.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                  ctypes.byref(rng), ctypes.byref(h))
        _check(st, "adk_mlp_create")
        self._h = h

    @classmethod
    def load(cls, gas: Gas, path: str):
        h = ctypes.c_void_p()
        _check(lib().adk_mlp_load(gas.handle, str(path).encode(), ctypes.byref(h)), "adk_mlp_load")
        return cls(gas, _handle=h)

    def save(self, path: str):
        _check(lib().adk_mlp_save(self._h, str(path).encode()), "adk_mlp_save")

    def state(self):
        """(params, m, v, step) as host float32 arrays and int."""
        p = np.empty(self.nparams, np.float32)
        m = np.empty(self.nparams, np.float32)
        v = np.empty(self.nparams, np.float32)
        step = ctypes.c_int64()
        st = lib().adk_mlp_get_state(self._h, p.ctypes.data_as(ctypes.c_void_p), m.ctypes.data_as(ctypes.c_void_p),
                                     v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(step))
        _check(st, "adk_mlp_get_state")
        return p, m, v, int(step.value)

    def forward(self, E, dt, k, stream=None):
        import torch
        n = E.numel()
        Q = torch.empty((4, n), dtype=torch.float32, device=E.device)
        st = lib().adk_mlp_forward(self._h, _dev(E, "E"), _dev(dt, "dt"), _dev(k, "k"), n, _dev(Q, "Q"),
                                   _stream(stream))
        _check(st, "adk_mlp_forward")
        return Q

    def loss_grad(self, E, dt, k, stream=None):
        import torch
        n = E.numel()
        g = torch.empty(self.nparams, dtype=torch.float32, device=E.device)
        L = torch.empty(1, dtype=torch.float32, device=E.device)
        st = lib().adk_mlp_loss_grad(self._h, self._gas.handle, _dev(E, "E"), _dev(dt, "dt"), _dev(k, "k"), n,
                                     _dev(g, "grad"), _dev(L, "loss"), _stream(stream))
        _check(st, "adk_mlp_loss_grad")
        return L, g

    def forward_trace(self, E, dt, k, stream=None):
        """(Q[4][n], Zt[n][196]): the forward pass with its float32
        pre-activations of layers 1-3 and logits (adk_mlp_forward_trace)."""
        import torch
        n = E.numel()
        Q = torch.empty((4, n), dtype=torch.float32, device=E.device)
        Zt = torch.empty((n, 196), dtype=torch.float32, device=E.device)
        st = lib().adk_mlp_forward_trace(self._h, _dev(E, "E"), _dev(dt, "dt"), _dev(k, "k"), n, _dev(Q, "Q"),
                                         _dev(Zt, "Zt"), _stream(stream))
        _check(st, "adk_mlp_forward_trace")
        return Q, Zt

    def loss_grad_noalloc(self, E, dt, k, grad, loss, stream=None):
        """adk_mlp_loss_grad_noalloc: loss and gradient into the caller's
        device tensors grad (float32[nparams]) and loss (float32[1]), with no
        allocation in the library (n <= ADK_MLP_NOALLOC_MAX_SAMPLES)."""
        import torch
        if grad.dtype != torch.float32 or grad.numel() != self.nparams or loss.dtype != torch.float32:
            raise ValueError("grad must be float32[nparams] and loss float32[1]")
        st = lib().adk_mlp_loss_grad_noalloc(self._h, self._gas.handle, _dev(E, "E"), _dev(dt, "dt"), _dev(k, "k"),
                                             E.numel(), _dev(grad, "grad"), _dev(loss, "loss"), _stream(stream))
        _check(st, "adk_mlp_loss_grad_noalloc")
        return loss, grad

    def train(self, iters: int, nsamples: int = 1_000_000, batch: int = 4096, lr: float = 3e-3,
              lr_min: float = 1e-5, total_iters: Optional[int] = None, seed: int = 1, stream=None) -> np.ndarray:
        """Adam steps on the analytic solver's columns; returns the batch losses."""
        cfg = _TrainCfg(int(nsamples), int(iters), int(total_iters or iters), int(batch), float(lr), float(lr_min),
                        int(seed) & 0xFFFFFFFFFFFFFFFF)
        out = np.zeros(max(1, int(iters)), np.float32)
        st = lib().adk_mlp_train(self._h, self._gas.handle, ctypes.byref(cfg), out.ctypes.data_as(ctypes.c_void_p),
                                 _stream(stream))
        _check(st, "adk_mlp_train")
        return out[: int(iters)]

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().adk_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def surrogate_step(gas: Gas, mlp: Mlp, E, dt: float, pops, lo, w: int = 3, eps: float = 1e-8, counters=None,
                   stream=None):
    """Surrogate form of the step, in place on float32 pops[(w+1)][n] and lo;
    counters: optional int64 device tensor of 2 entries (see adk_surrogate_step)."""
    import torch
    n = E.numel()
    if E.dtype != torch.float32 or pops.dtype != torch.float32 or tuple(pops.shape) != (w + 1, n):
        raise ValueError(f"E float32[{n}] and pops float32[{w + 1}][{n}] expected")
    if lo.dtype != torch.uint8 or lo.numel() != n:
        raise ValueError("lo must be uint8[ncells]")
    cptr = None
    if counters is not None:
        if counters.dtype != torch.int64 or counters.numel() != 2:
            raise ValueError("counters must be int64[2]")
        cptr = _dev(counters, "counters")
    win = _Window(int(w), float(eps), ADK_LAYOUT_COMPACT, ADK_MIXED)
    st = lib().adk_surrogate_step(gas.handle, mlp.handle, _dev(E, "E"), n, float(dt), _dev(pops, "pops"),
                                  _dev(lo, "lo"), ctypes.byref(win), cptr, _stream(stream))
    _check(st, "adk_surrogate_step")
    return pops, lo
