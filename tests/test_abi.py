"""C ABI checks that need no GPU: the library loads, exports every function
that include/strom.h declares, and rejects invalid arguments on the host
before any launch."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1910_01260_amd import strom

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "strom.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(st_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("st_build_bases", "st_assemble", "st_solve", "st_form", "st_strerror", "st_rom_layout"):
        assert n in names


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", strom.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(ln.split()[-1] for ln in out.stdout.splitlines() if ln.strip())
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    lib = strom.lib()
    for n in declared_functions():
        assert hasattr(lib, n)


def test_binding_names_match_header():
    assert set(strom.EXPORTED) <= set(declared_functions())


def test_strerror_and_version():
    assert strom.st_version() == 2
    assert "workspace" in strom.st_strerror(-3)
    assert strom.st_strerror(12345) == "unknown status"


def test_layout_is_deterministic_and_aligned():
    d = strom.RomDesc([3, 5, 2], 10, 2, 1, 1)
    lay = strom.st_rom_layout(d)
    keys = ["Ahat", "bhat", "u0hat", "T", "K", "Wf", "P1", "mode", "moff", "koff", "Phit", "dt", "T32", "Tcn", "Au0",
            "total"]
    offs = [lay[k] for k in keys]
    assert offs == sorted(offs) and all(o % 256 == 0 for o in offs)
    n = 10
    assert lay["K"] - lay["T"] >= 8 * n * n
    assert lay["dt"] - lay["Phit"] >= 8 * 10 * n and lay["T32"] - lay["dt"] >= 8 * 10
    assert lay["Tcn"] - lay["T32"] >= 4 * n * n and lay["total"] == lay["Tcn"]     # backward Euler: no CN sections


def _null():
    return ctypes.c_void_p(0)


def test_host_validation_rejects_bad_arguments():
    L = strom.lib()
    good = strom.RomDesc([4, 4], 8, 2, 0, 1)
    bad_nt = strom.RomDesc([4, 9], 8, 2, 0, 1)      # n_t > N_t
    bad_q = strom.RomDesc([4, 4], 8, 0, 0, 1)       # Q = 0
    lay = strom.st_rom_layout_t()
    assert L.st_rom_layout(bad_nt.ref(), ctypes.byref(lay)) == -1
    assert L.st_rom_layout(bad_q.ref(), ctypes.byref(lay)) == -1
    assert L.st_rom_layout(None, ctypes.byref(lay)) == -1
    # st_solve: null rom, negative n_q, bad precision, bad tolerance
    fake = ctypes.c_void_p(0x1000)
    args = lambda **kw: dict(dict(d=good.ref(), rom=fake, n_q=4, thA=fake, thf=None, th0=fake, nt=None, prec=0,
                                  tol=0.0, irmax=0, coeff=fake, cap=100, coff=fake, relres=fake, info=fake,
                                  iters=None, ws=fake, wsb=1 << 20, stream=None), **kw)

    def call(a):
        return L.st_solve(a["d"], a["rom"], a["n_q"], a["thA"], a["thf"], a["th0"], a["nt"], None, a["prec"], a["tol"],
                          a["irmax"], a["coeff"], a["cap"], a["coff"], a["relres"], a["info"], a["iters"], a["ws"],
                          a["wsb"], a["stream"])

    assert call(args(rom=None)) == -1
    assert call(args(n_q=-1)) == -1
    assert call(args(prec=7)) == -1
    assert call(args(tol=-1.0)) == -1
    assert call(args(irmax=-2)) == -1
    assert call(args(thA=None)) == -1
    assert call(args(th0=None)) == -1                # Q0 = 1 needs theta_0
    assert call(args(coeff=None)) == -1
    assert call(args(wsb=16)) == -3                  # workspace too small
    assert call(args(d=bad_nt.ref())) == -1
    assert call(args(n_q=0)) == 0                    # empty batch: no-op, no launch
    # st_form: bad output precision
    assert L.st_form(good.ref(), fake, 4, fake, None, fake, None, 5, fake, 10, fake, 10, fake, fake, fake, fake,
                     1 << 20, None) == -1
    # st_assemble: rank and CSR shape checks
    csr = (strom.st_csr * 2)(strom.st_csr(16, 0, 0x1000, 0, 0), strom.st_csr(16, 0, 0x1000, 0, 0))
    assert L.st_assemble(good.ref(), 1, fake, fake, fake, csr, None, None, fake, 0, fake, 1 << 20, fake, 1 << 20,
                         None) == -4                 # n_s = 2 > N_s = 1
    assert L.st_assemble(good.ref(), 8, fake, fake, fake, csr, None, None, fake, 0, fake, 1 << 20, fake, 1 << 20,
                         None) == -1                 # CSR rows 16 != N_s 8
    assert L.st_assemble(good.ref(), 16, fake, fake, fake, csr, None, None, fake, 9, fake, 1 << 20, fake, 1 << 20,
                         None) == -1                 # bad projection precision


def test_workspace_sizes_with_empty_term_lists():
    """Zero input or initial-state terms must size cleanly on the host."""
    L = strom.lib()
    for Qf, Q0 in ((0, 0), (0, 1), (1, 0), (3, 2)):
        d = strom.RomDesc([8] * 8, 128, 2, Qf, Q0)
        assert L.st_assemble_workspace(d.ref(), 256) >= 2 * 8 * 256 * 8
        assert L.st_form_workspace(d.ref(), 10) > 0
        assert L.st_solve_workspace(d.ref(), 10, 640, 40960, 0) > 40960 * 8


def test_mlp_and_certificate_host_validation():
    """Surrogate entry points reject bad shapes and arguments before any launch."""
    L = strom.lib()
    fake = ctypes.c_void_p(0x1000)
    ok = strom.mlp_shape(3, 512, 4, 1200)
    assert strom.st_mlp_param_count(ok) == 3 * 512 + 512 + 3 * (512 * 512 + 512) + 512 * 1200 + 1200
    assert L.st_mlp_workspace(ctypes.byref(ok), 4096) > 4096 * 1200 * 4
    for bad in (strom.mlp_shape(0, 8, 1, 1), strom.mlp_shape(3, 8, 0, 1), strom.mlp_shape(3, 8, 1, 0),
                strom.mlp_shape(3, 8, 63, 1)):
        assert L.st_mlp_param_count(ctypes.byref(bad)) < 0
        assert L.st_mlp_workspace(ctypes.byref(bad), 10) == 0
        assert L.st_mlp_forward(ctypes.byref(bad), fake, 10, fake, fake, fake, 1 << 30, None) == -1
    assert L.st_mlp_forward(None, fake, 10, fake, fake, fake, 1 << 30, None) == -1
    # batch 0 is a no-op; null buffers and short workspaces are rejected
    assert L.st_mlp_forward(ctypes.byref(ok), None, 0, None, None, None, 0, None) == 0
    assert L.st_mlp_forward(ctypes.byref(ok), fake, 10, None, fake, fake, 1 << 30, None) == -1
    assert L.st_mlp_forward(ctypes.byref(ok), fake, 10, fake, fake, fake, 16, None) == -3
    assert L.st_mlp_grad(ctypes.byref(ok), fake, 0, fake, fake, fake, fake, fake, 1 << 30, None) == -1
    assert L.st_mlp_grad(ctypes.byref(ok), fake, 10, fake, fake, fake, fake, fake, 16, None) == -3
    f = ctypes.c_float
    assert L.st_mlp_adam(10, fake, fake, fake, fake, 0, f(1e-3), f(0.9), f(0.999), f(1e-8), None) == -1
    assert L.st_mlp_adam(10, fake, fake, fake, fake, 1, f(1e-3), f(1.0), f(0.999), f(1e-8), None) == -1
    assert L.st_mlp_adam(10, fake, fake, fake, fake, 1, f(1e-3), f(0.9), f(0.999), f(0.0), None) == -1
    assert L.st_mlp_adam(0, None, None, None, None, 1, f(1e-3), f(0.9), f(0.999), f(1e-8), None) == 0
    # certificate: gamma must be positive, tolerance non-negative
    d = strom.RomDesc([4, 4], 8, 2, 0, 1)
    nb = L.st_surrogate_check_workspace(d.ref(), 4)
    assert nb > 0
    call = lambda gamma, tol, ws=nb: L.st_surrogate_check(d.ref(), fake, 4, fake, None, fake, fake, fake, fake,
                                                         gamma, tol, fake, fake, fake, fake, ws, None)
    assert call(0.0, 1e-6) == -1
    assert call(1e-3, -1.0) == -1
    assert call(float("nan"), 1e-6) == -1
    assert call(1e-3, 1e-6, ws=nb - 1) == -3


def test_graph_and_autotune_host_calls():
    L = strom.lib()
    assert L.st_graph_enable(0) == 0
    assert L.st_graph_reset() == 0
    assert L.st_graph_count() == 0
    assert L.st_autotune_choice(7, 100) == -1           # bad precision
    assert L.st_autotune_choice(0, 1 << 20) == -1       # width out of range
    assert L.st_autotune_set(1, 100, 3) == -1           # no such variant
    assert L.st_autotune_set(1, 2000, 2) == -1          # the 256-thread variant is for widths <= 1536
    assert L.st_autotune_set(1, 100, 2) == 0
    assert L.st_autotune_set(1, 100, -1) == 0
    assert L.st_autotune_set(1, 100, 1) == 0
    assert L.st_autotune_choice(1, 100) == 1
    assert L.st_autotune_set(1, 100, -1) == 0
    assert L.st_autotune_choice(1, 100) == -1
    d = strom.RomDesc([4, 4], 8, 2, 0, 1)
    fake = ctypes.c_void_p(0x1000)
    # bad precision and short workspace are rejected before any launch
    assert L.st_autotune(d.ref(), fake, 4, fake, None, fake, None, 5, fake, 100, fake, fake, fake, fake, 1 << 30,
                         None, None, None) == -1
    assert L.st_autotune(d.ref(), fake, 4, fake, None, fake, None, 1, fake, 100, fake, fake, fake, fake, 16,
                         None, None, None) == -3
