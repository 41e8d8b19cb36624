"""ctypes binding of libstrom.so (the gfx950 ST-ROM library).

Functions carry the C ABI's names and only marshal arguments: torch device
tensors are passed as raw pointers, outputs and workspaces are allocated with
torch (device memory plumbing), and the current torch stream is handed to the
library.  Every computation runs in the library's HIP kernels; if the library
is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstrom.so")

ST_F64, ST_F32, ST_BF16X3 = 0, 1, 2
ST_BACKWARD_EULER, ST_CRANK_NICOLSON = 0, 1
ST_OK = 0


class StromError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {st_strerror(code)} (status {code})")
        self.code = code


class st_csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class st_rom_desc(ctypes.Structure):
    _fields_ = [("n_s", ctypes.c_int32), ("N_t", ctypes.c_int32), ("Q", ctypes.c_int32), ("Qf", ctypes.c_int32),
                ("Q0", ctypes.c_int32), ("n_t", ctypes.POINTER(ctypes.c_int32)), ("integrator", ctypes.c_int32)]


class st_rom_layout_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_size_t) for k in ("Ahat", "bhat", "u0hat", "T", "K", "Wf", "P1", "mode", "moff", "koff", "Phit", "dt",
                                               "T32", "Tcn", "Au0", "total")]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_D = ctypes.c_double

_SIGNATURES = {
    "st_strerror": (ctypes.c_char_p, [_I32]),
    "st_version": (_I32, []),
    "st_rom_layout": (_I32, [ctypes.POINTER(st_rom_desc), ctypes.POINTER(st_rom_layout_t)]),
    "st_build_bases_workspace": (_SZ, [_I64, _I32, _I32, _I32, _P, _I32]),
    "st_build_bases": (_I32, [_P, _I32, _I64, _I64, _I32, _I32, _I32, _P, _I32, _D, _P, _P, _P, _P, _P, _P, _SZ,
                              _P]),
    "st_assemble_workspace": (_SZ, [ctypes.POINTER(st_rom_desc), _I64]),
    "st_assemble": (_I32, [ctypes.POINTER(st_rom_desc), _I64, _P, _P, _P, ctypes.POINTER(st_csr), _P, _P, _P, _I32, _P,
                           _SZ, _P, _SZ, _P]),
    "st_form_workspace": (_SZ, [ctypes.POINTER(st_rom_desc), _I32]),
    "st_form": (_I32, [ctypes.POINTER(st_rom_desc), _P, _I32, _P, _P, _P, _P, _I32, _P, _I64, _P, _I64, _P, _P, _P,
                       _P, _SZ, _P]),
    "st_solve_workspace": (_SZ, [ctypes.POINTER(st_rom_desc), _I32, _I64, _I64, _I32]),
    "st_solve": (_I32, [ctypes.POINTER(st_rom_desc), _P, _I32, _P, _P, _P, _P, _P, _I32, _D, _I32, _P, _I64, _P, _P,
                        _P, _P, _P, _SZ, _P]),
    "st_solve_noalloc": (_I32, [ctypes.POINTER(st_rom_desc), _P, _I32, _P, _P, _P, _P, _P, _I32, _D, _I32, _P, _I64,
                                _P, _P, _P, _P, _P]),
    "st_reconstruct": (_I32, [ctypes.POINTER(st_rom_desc), _P, _I64, _P, _I64, _P, _I64, _I32, _P, _P, _P, _P, _I64,
                              _P]),
    "st_graph_enable": (_I32, [_I32]),
    "st_graph_reset": (_I32, []),
    "st_graph_count": (_I32, []),
    "st_autotune": (_I32, [ctypes.POINTER(st_rom_desc), _P, _I32, _P, _P, _P, _P, _I32, _P, _I64, _P, _P, _P, _P,
                           _SZ, _P, _P, _P]),
    "st_autotune_choice": (_I32, [_I32, _I32]),
    "st_autotune_set": (_I32, [_I32, _I32, _I32]),
    "st_mlp_param_count": (_I64, [_P]),
    "st_mlp_workspace": (_SZ, [_P, _I32]),
    "st_mlp_forward": (_I32, [_P, _P, _I32, _P, _P, _P, _SZ, _P]),
    "st_mlp_grad": (_I32, [_P, _P, _I32, _P, _P, _P, _P, _P, _SZ, _P]),
    "st_mlp_adam": (_I32, [_I64, _P, _P, _P, _P, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           _P]),
    "st_mlp_colstats": (_I32, [_I32, _I32, _P, _P, _P, _P]),
    "st_mlp_standardize": (_I32, [_I32, _I32, _P, _P, _P, _P, _P]),
    "st_surrogate_check_workspace": (_SZ, [ctypes.POINTER(st_rom_desc), _I32]),
    "st_surrogate_check": (_I32, [ctypes.POINTER(st_rom_desc), _P, _I32, _P, _P, _P, _P, _P, _P, _D, _D, _P, _P, _P,
                                  _P, _SZ, _P]),
    "st_coercivity_floor": (_D, [_I32]),
    "st_certify_workspace": (_SZ, [ctypes.POINTER(st_rom_desc), _I32, _I64]),
    "st_certify": (_I32, [ctypes.POINTER(st_rom_desc), _P, _I32, _P, _P, _P, _P, _P, _I64, _D, _P, _P, _P, _SZ, _P]),
    "st_fom_bound_workspace": (_SZ, [ctypes.POINTER(st_rom_desc), _I64, _I32]),
    "st_fom_bound": (_I32, [ctypes.POINTER(st_rom_desc), _P, _I64, _P, ctypes.POINTER(st_csr), _P, _P, _P, _I32, _P,
                            _P, _P, _P, _P, _I64, _D, _P, _P, _P, _P, _SZ, _P]),
    "st_spatial_march": (_I32, [ctypes.POINTER(st_rom_desc), _P, _I32, _P, _P, _P, _P, _I32, _P, _P, _P, _P, _P]),
    "st_project_workspace": (_SZ, [_I64, _I32, _I32]),
    "st_project": (_I32, [_I64, _I32, _P, _I32, _P, _P, _P, _SZ, _P]),
    "st_gram_workspace": (_SZ, [_I64, _I32]),
    "st_gram": (_I32, [_P, _I32, _I64, _I64, _I32, _I32, _P, _P, _SZ, _P]),
    "st_isvd_workspace": (_SZ, [_I64, _I32]),
    "st_isvd_reset": (_I32, [_P, _P]),
    "st_isvd_update": (_I32, [_P, _I64, _I64, _I32, _I32, _I64, _D, _D, _P, _P, _P, _P, _P, _SZ, _P]),
    "st_isvd_bases_workspace": (_SZ, [_I32, _I32, _I32]),
    "st_isvd_bases": (_I32, [_P, _P, _P, _P, _I64, _I64, _I32, _I32, _I32, _P, _D, _P, _P, _P, _P, _P, _SZ, _P]),
    "st_timing_enable": (_I32, [_I32]),
    "st_timing_read": (_I32, [ctypes.POINTER(ctypes.c_double), _I32]),
}

TIMING_PHASES = ("plan", "form", "rhs_norms", "lu", "first_solve", "refinement", "final_check")

EXPORTED = tuple(_SIGNATURES)


def lib():
    """Load libstrom.so once; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libstrom.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def st_strerror(code: int) -> str:
    return lib().st_strerror(int(code)).decode()


def st_version() -> int:
    return int(lib().st_version())


def _check(code: int, where: str):
    if code != ST_OK:
        raise StromError(code, where)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _colptr(t: torch.Tensor):
    """Pointer of a column-major device matrix (unit stride down a column; any leading dimension)."""
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dim() != 2 or t.stride(0) != 1 or t.stride(1) < t.shape[0]:
        raise ValueError("expected a column-major matrix")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class RomDesc:
    """Host description of a reduced model (keeps its n_t array alive)."""

    def __init__(self, n_t: Sequence[int], N_t: int, Q: int, Qf: int, Q0: int, integrator: int = 0):
        self.n_t_arr = np.ascontiguousarray(np.asarray(n_t, dtype=np.int32))
        self.n_t_ptr = self.n_t_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.c = st_rom_desc(len(self.n_t_arr), int(N_t), int(Q), int(Qf), int(Q0), self.n_t_ptr, int(integrator))

    @property
    def N_t(self):
        return int(self.c.N_t)

    @property
    def n_t(self):
        return self.n_t_arr.tolist()

    @property
    def n_s(self):
        return int(self.c.n_s)

    @property
    def n(self):
        return int(self.n_t_arr.sum())

    def ref(self):
        return ctypes.byref(self.c)


def st_rom_layout(desc: RomDesc) -> dict:
    out = st_rom_layout_t()
    _check(lib().st_rom_layout(desc.ref(), ctypes.byref(out)), "st_rom_layout")
    return {k: int(getattr(out, k)) for k, _ in st_rom_layout_t._fields_}


def csr_to_device(row_ptr, col_idx, val, device="cuda"):
    """Device copies of CSR arrays (int32, int32, float64) and their descriptor."""
    rp = torch.as_tensor(np.asarray(row_ptr, dtype=np.int32), device=device)
    ci = torch.as_tensor(np.asarray(col_idx, dtype=np.int32), device=device)
    va = torch.as_tensor(np.asarray(val, dtype=np.float64), device=device)
    d = st_csr(int(rp.numel() - 1), int(ci.numel()), rp.data_ptr(), ci.data_ptr(), va.data_ptr())
    return d, (rp, ci, va)


POD_DIAG = ("ritz_residual", "jacobi_sweeps", "jacobi_off", "refine_cols", "jacobi_fallback_sweeps")


def st_build_bases(U: torch.Tensor, N_t: int, n_mu: int, n_s: int, n_t: Sequence[int], gram_prec: int = ST_F64,
                   tau_t: float = 1e-7, diag: Optional[torch.Tensor] = None):
    """POD on the device.  U: (N_s, n_mu*N_t) column-major, i.e. a tensor whose
    transpose is contiguous (pass U.T.contiguous().T or torch.empty((m, N_s)).T).
    diag: optional device float64 tensor of len(POD_DIAG) receiving the
    convergence diagnostics.
    Returns (Phi_s (N_s x n_s, column-major view), Phi_t (N_t x n), sigma, rank_t)."""
    N_s = U.shape[0]
    if U.T.is_contiguous():
        ld = U.stride(1)
    else:
        raise ValueError("U must be column-major (U.T contiguous)")
    prec = ST_F64 if U.dtype == torch.float64 else ST_F32
    if diag is not None and (diag.dtype != torch.float64 or diag.device != U.device or not diag.is_contiguous()
                             or diag.numel() < len(POD_DIAG)):
        raise ValueError(f"diag must be a contiguous float64 tensor of >= {len(POD_DIAG)} elements on U's device")
    nt = np.ascontiguousarray(np.asarray(n_t, dtype=np.int32))
    n = int(nt.sum())
    ws_bytes = lib().st_build_bases_workspace(N_s, N_t, n_mu, n_s, nt.ctypes.data, gram_prec)
    if ws_bytes == 0:
        raise StromError(-1, "st_build_bases_workspace")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=U.device)
    Phi_s = torch.empty((n_s, N_s), dtype=torch.float64, device=U.device)
    Phi_t = torch.empty((n, N_t), dtype=torch.float64, device=U.device)
    sigma = torch.empty(n_s, dtype=torch.float64, device=U.device)
    rank = torch.empty(n_s, dtype=torch.int32, device=U.device)
    _check(lib().st_build_bases(ctypes.c_void_p(U.data_ptr()), prec, ld, N_s, N_t, n_mu, n_s, nt.ctypes.data, gram_prec,
                                float(tau_t), _ptr(Phi_s), _ptr(Phi_t), _ptr(sigma), _ptr(rank), _ptr(diag), _ptr(ws),
                                ws_bytes,
                                _stream()), "st_build_bases")
    return Phi_s.T, Phi_t.T, sigma, rank


def st_assemble(desc: RomDesc, Phi_s: torch.Tensor, Phi_t: torch.Tensor, dt: torch.Tensor, A_csr: list,
                Bf: Optional[torch.Tensor] = None, g: Optional[torch.Tensor] = None,
                u0: Optional[torch.Tensor] = None, proj_prec: int = ST_F64) -> torch.Tensor:
    """Offline ROM buffer.  Phi_s (N_s x n_s) and Phi_t (N_t x n) column-major
    (transposes contiguous); Bf (N_s x Qf), g (N_t x Qf), u0 (N_s x Q0)
    column-major likewise; A_csr a list of st_csr descriptors."""
    N_s = Phi_s.shape[0]

    def colmajor(t):
        if t is None:
            return None
        if not t.T.is_contiguous():
            raise ValueError("expected a column-major tensor (transpose contiguous)")
        return ctypes.c_void_p(t.data_ptr())

    lay = st_rom_layout(desc)
    rom = torch.empty(lay["total"], dtype=torch.uint8, device=Phi_s.device)
    ws_bytes = lib().st_assemble_workspace(desc.ref(), N_s)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=Phi_s.device)
    arr = (st_csr * len(A_csr))(*A_csr)
    _check(lib().st_assemble(desc.ref(), N_s, colmajor(Phi_s), colmajor(Phi_t), _ptr(dt), arr, colmajor(Bf),
                             colmajor(g), colmajor(u0), int(proj_prec), _ptr(rom), lay["total"], _ptr(ws), ws_bytes,
                             _stream()),
           "st_assemble")
    return rom


def rom_section(desc: RomDesc, rom: torch.Tensor, name: str) -> torch.Tensor:
    """View of one FP64 section of a ROM buffer (flat)."""
    lay = st_rom_layout(desc)
    order = ["Ahat", "bhat", "u0hat", "T", "K", "Wf", "P1", "mode", "moff", "koff", "Phit", "dt", "T32", "Tcn", "Au0",
             "total"]
    i = order.index(name)
    b0, b1 = lay[name], lay[order[i + 1]]
    dtype = {"mode": torch.int32, "moff": torch.int32, "koff": torch.int64, "T32": torch.float32}.get(name,
                                                                                                    torch.float64)
    return rom[b0:b1].view(dtype)


def query_widths(desc: RomDesc, nt_q: Optional[np.ndarray], n_q: int) -> np.ndarray:
    if nt_q is None:
        return np.full(n_q, desc.n, dtype=np.int64)
    return np.asarray(nt_q, dtype=np.int64).sum(axis=1)


def st_form(desc: RomDesc, rom: torch.Tensor, theta_A: torch.Tensor, theta_f: Optional[torch.Tensor] = None,
            theta_0: Optional[torch.Tensor] = None, nt_q: Optional[torch.Tensor] = None, out_prec: int = ST_F64,
            widths: Optional[np.ndarray] = None):
    """Per-query reduced systems.  Returns (mats flat, rhs, coeff_off, mat_off, info)."""
    n_q = int(theta_A.shape[0])
    dev = theta_A.device
    if widths is None:
        widths = query_widths(desc, None if nt_q is None else nt_q.cpu().numpy(), n_q)
    sum_w = int(widths.sum())
    sum_w2 = int((widths.astype(np.int64) ** 2).sum())
    mats = torch.empty(max(sum_w2, 1), dtype=torch.float64 if out_prec == ST_F64 else torch.float32, device=dev)
    rhs = torch.empty(max(sum_w, 1), dtype=torch.float64, device=dev)
    coeff_off = torch.empty(n_q + 1, dtype=torch.int64, device=dev)
    mat_off = torch.empty(n_q + 1, dtype=torch.int64, device=dev)
    info = torch.empty(max(n_q, 1), dtype=torch.int32, device=dev)
    ws_bytes = lib().st_form_workspace(desc.ref(), n_q)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    _check(lib().st_form(desc.ref(), _ptr(rom), n_q, _ptr(theta_A), _ptr(theta_f), _ptr(theta_0), _ptr(nt_q),
                         out_prec, _ptr(mats), sum_w2, _ptr(rhs), sum_w, _ptr(coeff_off), _ptr(mat_off), _ptr(info),
                         _ptr(ws), ws_bytes, _stream()), "st_form")
    return mats, rhs, coeff_off, mat_off, info[:n_q]


class SolveBuffers:
    """Preallocated outputs and workspace of st_solve for a fixed query mix."""

    def __init__(self, desc: RomDesc, n_q: int, widths: np.ndarray, lu_prec: int, device="cuda"):
        self.n_q = n_q
        self.sum_w = int(widths.sum())
        self.sum_w2 = int((widths.astype(np.int64) ** 2).sum())
        self.lu_prec = lu_prec
        self.coeff = torch.empty(max(self.sum_w, 1), dtype=torch.float64, device=device)
        self.coeff_off = torch.empty(n_q + 1, dtype=torch.int64, device=device)
        self.relres = torch.empty(max(n_q, 1), dtype=torch.float64, device=device)
        self.info = torch.empty(max(n_q, 1), dtype=torch.int32, device=device)
        self.iters = torch.empty(max(n_q, 1), dtype=torch.int32, device=device)
        self.ws_bytes = lib().st_solve_workspace(desc.ref(), n_q, self.sum_w, self.sum_w2, lu_prec)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)


def st_solve(desc: RomDesc, rom: torch.Tensor, theta_A: torch.Tensor, theta_f: Optional[torch.Tensor] = None,
             theta_0: Optional[torch.Tensor] = None, nt_q: Optional[torch.Tensor] = None, lu_prec: int = ST_F64,
             ir_tol: float = 0.0, ir_max: int = 0, bufs: Optional[SolveBuffers] = None,
             widths: Optional[np.ndarray] = None, skip: Optional[torch.Tensor] = None) -> SolveBuffers:
    """Batched reduced solve; returns the SolveBuffers holding coeff, coeff_off,
    relres, info, iters."""
    n_q = int(theta_A.shape[0])
    if bufs is None:
        if widths is None:
            widths = query_widths(desc, None if nt_q is None else nt_q.cpu().numpy(), n_q)
        bufs = SolveBuffers(desc, n_q, widths, lu_prec, theta_A.device)
    _check(lib().st_solve(desc.ref(), _ptr(rom), n_q, _ptr(theta_A), _ptr(theta_f), _ptr(theta_0), _ptr(nt_q),
                          _ptr(skip), lu_prec, float(ir_tol), int(ir_max), _ptr(bufs.coeff), bufs.sum_w, _ptr(bufs.coeff_off),
                          _ptr(bufs.relres), _ptr(bufs.info), _ptr(bufs.iters), _ptr(bufs.ws), bufs.ws_bytes,
                          _stream()), "st_solve")
    return bufs


NOALLOC_SCRATCH_BYTES = 64 << 20


def st_solve_noalloc(desc: RomDesc, rom: torch.Tensor, theta_A: torch.Tensor, theta_f: Optional[torch.Tensor] = None,
                     theta_0: Optional[torch.Tensor] = None, nt_q: Optional[torch.Tensor] = None,
                     lu_prec: int = ST_F64, ir_tol: float = 0.0, ir_max: int = 0, bufs: Optional[SolveBuffers] = None,
                     widths: Optional[np.ndarray] = None, skip: Optional[torch.Tensor] = None) -> SolveBuffers:
    """st_solve with the library's static workspace (no workspace argument).
    Output buffers as st_solve's (bufs.ws is not used)."""
    n_q = int(theta_A.shape[0])
    if bufs is None:
        if widths is None:
            widths = query_widths(desc, None if nt_q is None else nt_q.cpu().numpy(), n_q)
        bufs = SolveBuffers(desc, n_q, widths, lu_prec, theta_A.device)
    _check(lib().st_solve_noalloc(desc.ref(), _ptr(rom), n_q, _ptr(theta_A), _ptr(theta_f), _ptr(theta_0), _ptr(nt_q),
                                  _ptr(skip), lu_prec, float(ir_tol), int(ir_max), _ptr(bufs.coeff), bufs.sum_w,
                                  _ptr(bufs.coeff_off), _ptr(bufs.relres), _ptr(bufs.info), _ptr(bufs.iters),
                                  _stream()), "st_solve_noalloc")
    return bufs


def st_reconstruct(desc: RomDesc, rom: torch.Tensor, Phi_s: torch.Tensor, Phi_t: torch.Tensor,
                   bufs: "SolveBuffers", n_q: int, nt_q: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Space-time states of the first n_q queries of a solve: (n_q, N_t, N_s) view of
    column-major N_s x N_t blocks (Phi_s, Phi_t column-major device tensors)."""
    N_s = int(Phi_s.shape[0])
    N_t = desc.c.N_t
    out = torch.empty((n_q, N_t, N_s), dtype=torch.float64, device=Phi_s.device)
    _check(lib().st_reconstruct(desc.ref(), _ptr(rom), N_s, _colptr(Phi_s), int(Phi_s.stride(1)), _colptr(Phi_t),
                                int(Phi_t.stride(1)), int(n_q), _ptr(nt_q), _ptr(bufs.coeff), _ptr(bufs.coeff_off),
                                _ptr(out), N_s, _stream()), "st_reconstruct")
    return out


def st_graph_enable(on: bool = True):
    _check(lib().st_graph_enable(1 if on else 0), "st_graph_enable")


def st_graph_reset():
    _check(lib().st_graph_reset(), "st_graph_reset")


def st_graph_count() -> int:
    return int(lib().st_graph_count())


LU_VARIANTS = 3


def st_autotune(desc: RomDesc, rom: torch.Tensor, theta_A: torch.Tensor, theta_f: Optional[torch.Tensor] = None,
                theta_0: Optional[torch.Tensor] = None, nt_q: Optional[torch.Tensor] = None, lu_prec: int = ST_F64,
                bufs: Optional[SolveBuffers] = None, widths: Optional[np.ndarray] = None):
    """Time the batched-LU variants on this batch and record the fastest.
    Returns (choice, [ms per variant]).  bufs' outputs are scratch afterwards."""
    n_q = int(theta_A.shape[0])
    if bufs is None:
        if widths is None:
            widths = query_widths(desc, None if nt_q is None else nt_q.cpu().numpy(), n_q)
        bufs = SolveBuffers(desc, n_q, widths, lu_prec, theta_A.device)
    choice = ctypes.c_int32(-1)
    ms = (ctypes.c_double * LU_VARIANTS)()
    _check(lib().st_autotune(desc.ref(), _ptr(rom), n_q, _ptr(theta_A), _ptr(theta_f), _ptr(theta_0), _ptr(nt_q),
                             lu_prec, _ptr(bufs.coeff), bufs.sum_w, _ptr(bufs.coeff_off), _ptr(bufs.relres),
                             _ptr(bufs.info), _ptr(bufs.ws), bufs.ws_bytes, _stream(), ctypes.byref(choice), ms),
           "st_autotune")
    return int(choice.value), [float(ms[i]) for i in range(LU_VARIANTS)]


def st_autotune_choice(lu_prec: int, n: int) -> int:
    return int(lib().st_autotune_choice(lu_prec, n))


def st_autotune_set(lu_prec: int, n: int, variant: int):
    _check(lib().st_autotune_set(lu_prec, n, variant), "st_autotune_set")


def st_timing_enable(on: bool = True):
    _check(lib().st_timing_enable(1 if on else 0), "st_timing_enable")


def st_timing_read() -> dict:
    """Phase durations (ms) of the most recent st_solve; the stream must be synchronised."""
    buf = (ctypes.c_double * len(TIMING_PHASES))()
    n = lib().st_timing_read(buf, len(TIMING_PHASES))
    if n < 0:
        raise StromError(n, "st_timing_read")
    return {k: float(buf[i]) for i, k in enumerate(TIMING_PHASES)}


# ----------------------------------------------------------------------------
# surrogate network
# ----------------------------------------------------------------------------

class st_mlp_shape(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_int32), ("width", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("d_out", ctypes.c_int32)]


def mlp_shape(d_in: int, width: int, n_hidden: int, d_out: int) -> st_mlp_shape:
    return st_mlp_shape(int(d_in), int(width), int(n_hidden), int(d_out))


def st_mlp_param_count(shape: st_mlp_shape) -> int:
    n = int(lib().st_mlp_param_count(ctypes.byref(shape)))
    if n < 0:
        raise StromError(-1, "st_mlp_param_count")
    return n


def _mlp_ws(shape, batch, device):
    nb = lib().st_mlp_workspace(ctypes.byref(shape), int(batch))
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device), nb


def st_mlp_forward(shape: st_mlp_shape, params: torch.Tensor, X: torch.Tensor, ws=None) -> torch.Tensor:
    batch = int(X.shape[0])
    Y = torch.empty((batch, shape.d_out), dtype=torch.float32, device=X.device)
    if ws is None:
        ws = _mlp_ws(shape, batch, X.device)
    _check(lib().st_mlp_forward(ctypes.byref(shape), _ptr(params), batch, _ptr(X), _ptr(Y), _ptr(ws[0]), ws[1],
                                _stream()), "st_mlp_forward")
    return Y


def st_mlp_grad(shape: st_mlp_shape, params: torch.Tensor, X: torch.Tensor, T: torch.Tensor, grads: torch.Tensor,
                loss: torch.Tensor, ws=None):
    batch = int(X.shape[0])
    if ws is None:
        ws = _mlp_ws(shape, batch, X.device)
    _check(lib().st_mlp_grad(ctypes.byref(shape), _ptr(params), batch, _ptr(X), _ptr(T), _ptr(grads), _ptr(loss),
                             _ptr(ws[0]), ws[1], _stream()), "st_mlp_grad")


def st_mlp_adam(params: torch.Tensor, grads: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
                beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    _check(lib().st_mlp_adam(int(params.numel()), _ptr(params), _ptr(grads), _ptr(m), _ptr(v), int(step), float(lr),
                             float(beta1), float(beta2), float(eps), _stream()), "st_mlp_adam")


def st_surrogate_check(desc: RomDesc, rom: torch.Tensor, theta_A: torch.Tensor, theta_f, theta_0, Y: torch.Tensor,
                       mean: torch.Tensor, scale: torch.Tensor, gamma: float, tol: float, coeff: torch.Tensor,
                       cert: torch.Tensor, accept: torch.Tensor):
    n_q = int(theta_A.shape[0])
    nb = lib().st_surrogate_check_workspace(desc.ref(), n_q)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=theta_A.device)
    _check(lib().st_surrogate_check(desc.ref(), _ptr(rom), n_q, _ptr(theta_A), _ptr(theta_f), _ptr(theta_0), _ptr(Y),
                                    _ptr(mean), _ptr(scale), float(gamma), float(tol), _ptr(coeff), _ptr(cert),
                                    _ptr(accept), _ptr(ws), nb, _stream()), "st_surrogate_check")


def st_coercivity_floor(N_t: int) -> float:
    return float(lib().st_coercivity_floor(int(N_t)))


def st_certify(desc: RomDesc, rom: torch.Tensor, theta_A: torch.Tensor, theta_f: Optional[torch.Tensor],
               theta_0: Optional[torch.Tensor], coeff: torch.Tensor, nt_q: Optional[torch.Tensor] = None,
               gamma: float = 0.0, coeff_cap: Optional[int] = None):
    """Per-query FP64 residual and relative-error certificate of packed
    coefficients.  Returns (relres, cert) device tensors of n_q entries."""
    n_q = int(theta_A.shape[0])
    dev = theta_A.device
    cap = int(coeff.numel()) if coeff_cap is None else int(coeff_cap)
    relres = torch.empty(max(n_q, 1), dtype=torch.float64, device=dev)
    cert = torch.empty(max(n_q, 1), dtype=torch.float64, device=dev)
    ws_bytes = lib().st_certify_workspace(desc.ref(), n_q, cap)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    _check(lib().st_certify(desc.ref(), _ptr(rom), n_q, _ptr(theta_A), _ptr(theta_f), _ptr(theta_0), _ptr(nt_q),
                            _ptr(coeff), cap, float(gamma), _ptr(relres), _ptr(cert), _ptr(ws), ws_bytes, _stream()),
           "st_certify")
    return relres[:n_q], cert[:n_q]


def st_fom_bound(desc: RomDesc, rom: torch.Tensor, Phi_s: torch.Tensor, A_csr: list, Bf: Optional[torch.Tensor],
                 g: Optional[torch.Tensor], u0: Optional[torch.Tensor], theta_A: torch.Tensor,
                 theta_f: Optional[torch.Tensor], theta_0: Optional[torch.Tensor], coeff: torch.Tensor,
                 nt_q: Optional[torch.Tensor] = None, inv_norm: float = 0.0, coeff_cap: Optional[int] = None):
    """Full-order space-time residual and Theorem-3 bound per query.  Phi_s, Bf, g,
    u0 column-major as for st_assemble.  Returns (res_inf, u_inf, bound)."""
    n_q = int(theta_A.shape[0])
    dev = theta_A.device
    N_s = int(Phi_s.shape[0])
    cap = int(coeff.numel()) if coeff_cap is None else int(coeff_cap)

    def colmajor(t):
        if t is None:
            return None
        if not t.T.is_contiguous():
            raise ValueError("expected a column-major tensor (transpose contiguous)")
        return ctypes.c_void_p(t.data_ptr())

    out = [torch.empty(max(n_q, 1), dtype=torch.float64, device=dev) for _ in range(3)]
    ws_bytes = lib().st_fom_bound_workspace(desc.ref(), N_s, n_q)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    arr = (st_csr * len(A_csr))(*A_csr)
    _check(lib().st_fom_bound(desc.ref(), _ptr(rom), N_s, colmajor(Phi_s), arr, colmajor(Bf), colmajor(g), colmajor(u0),
                              n_q, _ptr(theta_A), _ptr(theta_f), _ptr(theta_0), _ptr(nt_q), _ptr(coeff), cap,
                              float(inv_norm), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(ws), ws_bytes,
                              _stream()), "st_fom_bound")
    return tuple(o[:n_q] for o in out)


def st_project(Phi_s: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """Phi_s^T X (n_s x k, column-major view) for column-major Phi_s (N_s x n_s) and X (N_s x k)."""
    N_s, n_s = int(Phi_s.shape[0]), int(Phi_s.shape[1])
    k = int(X.shape[1])
    if not (Phi_s.T.is_contiguous() and X.T.is_contiguous()):
        raise ValueError("expected column-major tensors (transpose contiguous)")
    out = torch.empty((k, n_s), dtype=torch.float64, device=Phi_s.device)
    ws_bytes = lib().st_project_workspace(N_s, n_s, k)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=Phi_s.device)
    _check(lib().st_project(N_s, n_s, ctypes.c_void_p(Phi_s.data_ptr()), k, ctypes.c_void_p(X.data_ptr()), _ptr(out),
                            _ptr(ws), ws_bytes, _stream()), "st_project")
    return out.T


def st_spatial_march(desc: RomDesc, rom: torch.Tensor, theta_A: torch.Tensor, theta_f: Optional[torch.Tensor],
                     theta_0: Optional[torch.Tensor], g: Optional[torch.Tensor] = None,
                     Chat: Optional[torch.Tensor] = None, want_traj: bool = True):
    """Batched spatial-ROM march.  g (N_t x Qf) and Chat (n_s x n_out) column-major.
    Returns (traj (n_q, N_t, n_s) or None, outputs (n_q, N_t, n_out) or None, info)."""
    n_q = int(theta_A.shape[0])
    dev = theta_A.device
    traj = torch.empty((n_q, desc.N_t, desc.n_s), dtype=torch.float64, device=dev) if want_traj else None
    n_out = int(Chat.shape[1]) if Chat is not None else 0
    outs = torch.empty((n_q, desc.N_t, n_out), dtype=torch.float64, device=dev) if Chat is not None else None
    info = torch.empty(max(n_q, 1), dtype=torch.int32, device=dev)

    def colmajor(t):
        if t is None:
            return None
        if not t.T.is_contiguous():
            raise ValueError("expected a column-major tensor (transpose contiguous)")
        return ctypes.c_void_p(t.data_ptr())

    _check(lib().st_spatial_march(desc.ref(), _ptr(rom), n_q, _ptr(theta_A), _ptr(theta_f), _ptr(theta_0), colmajor(g),
                                  n_out, colmajor(Chat), _ptr(traj), _ptr(outs), _ptr(info), _stream()),
           "st_spatial_march")
    return traj, outs, info[:n_q]


ISVD_STATE = 16
ISVD_MAX_RANK = 256
ISVD_STATE_NAMES = ("rank", "snapshots", "reorthonormalisations", "dependent", "truncated", "skipped", "refused")


class IncrementalSVD:
    """Device buffers of one incremental-SVD stream (st_isvd_*): W (N_s x r_max),
    s (r_max), V (m_max x r_max), the state words and the workspace."""

    def __init__(self, N_s: int, r_max: int, m_max: int, eps_svd: float, eps_sv: float, device="cuda"):
        self.N_s, self.r_max, self.m_max = int(N_s), int(r_max), int(m_max)
        self.eps_svd, self.eps_sv = float(eps_svd), float(eps_sv)
        self.W_store = torch.zeros((self.r_max, self.N_s), dtype=torch.float64, device=device)
        self.s = torch.zeros(self.r_max, dtype=torch.float64, device=device)
        self.V_store = torch.zeros((self.r_max, self.m_max), dtype=torch.float64, device=device)
        self.state = torch.zeros(ISVD_STATE, dtype=torch.int32, device=device)
        nb = lib().st_isvd_workspace(self.N_s, self.r_max)
        if nb == 0:
            raise StromError(-1, "st_isvd_workspace")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        self.reset()

    def reset(self):
        _check(lib().st_isvd_reset(_ptr(self.state), _stream()), "st_isvd_reset")

    def update(self, U: torch.Tensor):
        """Stream the columns of U (N_s x b, column-major, or one vector)."""
        if U.shape[0] != self.N_s or U.dtype != torch.float64 or not U.is_cuda:
            raise ValueError("U must be a float64 device tensor with N_s rows")
        if U.dim() == 1:
            U = U.contiguous()
            ptr, ld, b = ctypes.c_void_p(U.data_ptr()), self.N_s, 1
        else:
            if U.stride(0) != 1:
                U = U.T.contiguous().T
            ptr, ld, b = ctypes.c_void_p(U.data_ptr()), max(U.stride(1), self.N_s), U.shape[1]
        _check(lib().st_isvd_update(ptr, ld, self.N_s, b, self.r_max, self.m_max, self.eps_svd, self.eps_sv,
                                    _ptr(self.W_store), _ptr(self.s), _ptr(self.V_store), _ptr(self.state),
                                    _ptr(self.ws), self.ws.numel(), _stream()), "st_isvd_update")

    def counters(self) -> dict:
        st = self.state.cpu().numpy()
        return {k: int(st[i]) for i, k in enumerate(ISVD_STATE_NAMES)}

    def factors(self):
        """(W N_s x r, s r, V k x r) as host arrays."""
        c = self.counters()
        r, k = c["rank"], c["snapshots"]
        W = self.W_store[:r].cpu().numpy().T.copy()
        V = self.V_store[:r, :k].cpu().numpy().T.copy()
        return W, self.s[:r].cpu().numpy().copy(), V

    def bases(self, N_t: int, n_mu: int, n_s: int, n_t: Sequence[int], tau_t: float = 1e-7):
        """st_isvd_bases: (Phi_s N_s x n_s, Phi_t N_t x n, sigma n_s, rank_t n_s), column-major views."""
        nt = np.ascontiguousarray(np.asarray(n_t, dtype=np.int32))
        n = int(nt.sum())
        dev = self.W_store.device
        nb = lib().st_isvd_bases_workspace(N_t, n_mu, n_s)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        Phi_s = torch.empty((n_s, self.N_s), dtype=torch.float64, device=dev)
        Phi_t = torch.empty((n, N_t), dtype=torch.float64, device=dev)
        sigma = torch.empty(n_s, dtype=torch.float64, device=dev)
        rank = torch.empty(n_s, dtype=torch.int32, device=dev)
        _check(lib().st_isvd_bases(_ptr(self.W_store), _ptr(self.s), _ptr(self.V_store), _ptr(self.state), self.N_s,
                                   self.m_max, N_t, n_mu, n_s, nt.ctypes.data, float(tau_t), _ptr(Phi_s),
                                   _ptr(Phi_t), _ptr(sigma), _ptr(rank), _ptr(ws), nb, _stream()), "st_isvd_bases")
        return Phi_s.T, Phi_t.T, sigma, rank


def st_gram(X: torch.Tensor, gram_prec: int = ST_F64) -> torch.Tensor:
    """G = X^T X (p x p, FP64) of a column-major K x p device matrix (float32 or
    float64), in the given arithmetic."""
    if X.dim() != 2 or X.stride(0) != 1:
        raise ValueError("X must be column-major (X.T contiguous)")
    K, p = X.shape
    prec = ST_F64 if X.dtype == torch.float64 else ST_F32
    nb = lib().st_gram_workspace(K, p)
    if nb == 0:
        raise StromError(-1, "st_gram_workspace")
    ws = torch.empty(nb, dtype=torch.uint8, device=X.device)
    G = torch.empty((p, p), dtype=torch.float64, device=X.device)
    _check(lib().st_gram(ctypes.c_void_p(X.data_ptr()), prec, max(X.stride(1), K), K, p, gram_prec, _ptr(G), _ptr(ws),
                         nb, _stream()), "st_gram")
    return G


def st_mlp_colstats(C: torch.Tensor):
    """(mean, scale) per column of the n x d row-major FP64 device matrix C."""
    C = C.contiguous()
    n, d = C.shape
    mean = torch.empty(d, dtype=torch.float64, device=C.device)
    scale = torch.empty(d, dtype=torch.float64, device=C.device)
    _check(lib().st_mlp_colstats(n, d, _ptr(C), _ptr(mean), _ptr(scale), _stream()), "st_mlp_colstats")
    return mean, scale


def st_mlp_standardize(C: torch.Tensor, mean: torch.Tensor, scale: torch.Tensor) -> torch.Tensor:
    """FP32 (C - mean) / scale of the n x d row-major FP64 device matrix C."""
    C = C.contiguous()
    n, d = C.shape
    T = torch.empty((n, d), dtype=torch.float32, device=C.device)
    _check(lib().st_mlp_standardize(n, d, _ptr(C), _ptr(mean), _ptr(scale), _ptr(T), _stream()), "st_mlp_standardize")
    return T
