"""C-ABI contract tests that need no GPU: the library loads, exports every symbol
include/dna.h declares, and rejects invalid calls before enqueuing anything."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dna.h")
LIB = os.path.join(ROOT, "paper_1301_3389_amd", "libdna.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_0-9]+\s*\*?\s*([A-Za-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdna.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19, names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/dna.h but not exported"


def test_binding_covers_header():
    from paper_1301_3389_amd import dna
    assert sorted(dna.EXPORTED) == declared_functions()


def test_status_strings(lib):
    f = lib.dna_status_string
    f.restype = ctypes.c_char_p
    for s in range(7):
        assert f(s).decode().startswith("DNA_")
    assert b"unknown" in f(99)


def test_workspace_bytes(lib):
    from paper_1301_3389_amd import dna
    o = dna.make_opts()
    ws = dna._lib_ws
    assert ws(0, 10, 10, ctypes.byref(o)) == 0
    assert ws(10, -1, 10, ctypes.byref(o)) == 0
    small = ws(8, 8, 2, ctypes.byref(o))
    big = ws(1024, 8192, 64, ctypes.byref(o))
    assert 0 < small < big
    # the fused path (R <= 64) keeps Q and Q-bar on chip: no pair of N x T buffers
    assert big < 2 * 1024 * 8192 * 4
    # the tiled fp32 path (R > 64) hands Q and Q-bar over in 2 * N * T floats
    assert ws(1024, 8192, 65, ctypes.byref(o)) >= 2 * 1024 * 8192 * 4
    # the unrolled adjoint reads both at any rank
    assert dna._lib_uws(1024, 8192, 64, ctypes.byref(o)) >= 2 * 1024 * 8192 * 4


def test_noalloc_rejects_oversized_problems_before_any_launch(lib):
    """dna_iterate_noalloc refuses a problem whose workspace exceeds its
    scratch array on the host, naming both sizes (no HIP call is made)."""
    from paper_1301_3389_amd import dna
    o = dna.make_opts()
    fake = ctypes.c_void_p(256)            # never dereferenced: the call returns first
    N, T, R = 4096, 32768, 512
    st = dna._lib_iterate_noalloc(fake, fake, fake, N, T, R, 1, ctypes.byref(o), None)
    assert st == 6, st                     # DNA_EUNSUPPORTED
    msg = dna._lib_last_error().decode()
    need = dna._lib_ws(N, T, R, ctypes.byref(o))
    assert str(need) in msg and str(64 << 20) in msg, msg
    assert dna._lib_iterate_noalloc(fake, fake, fake, 8, 8, 2, -1, ctypes.byref(o), None) == 1
    assert dna._lib_iterate_noalloc(None, fake, fake, 8, 8, 2, 1, ctypes.byref(o), None) == 1


def test_invalid_arguments_rejected_before_launch():
    from paper_1301_3389_amd import dna
    o = dna.make_opts()
    fake = ctypes.c_void_p(0x1000)     # never dereferenced: validation fails first
    ws = ctypes.c_void_p(0x100000)
    null = ctypes.c_void_p(0)
    E = dna._lib_update_H
    # null data pointer
    assert E(null, fake, fake, 8, 8, 2, ctypes.byref(o), ws, 1 << 30, null, null, null, null) == 1
    # bad sizes
    assert E(fake, fake, fake, 0, 8, 2, ctypes.byref(o), ws, 1 << 30, null, null, null, null) == 1
    assert E(fake, fake, fake, 8, 8, -3, ctypes.byref(o), ws, 1 << 30, null, null, null, null) == 1
    # workspace too small
    assert E(fake, fake, fake, 8, 8, 2, ctypes.byref(o), ws, 16, null, null, null, null) == 2
    # misaligned workspace
    assert E(fake, fake, fake, 8, 8, 2, ctypes.byref(o), ctypes.c_void_p(0x100004), 1 << 30,
             null, null, null, null) == 1
    # bad options
    bad = dna.make_opts(eps=2.0)
    assert E(fake, fake, fake, 8, 8, 2, ctypes.byref(bad), ws, 1 << 30, null, null, null, null) == 1
    bad = dna.make_opts(alpha=-1.0)
    assert E(fake, fake, fake, 8, 8, 2, ctypes.byref(bad), ws, 1 << 30, null, null, null, null) == 1
    assert dna._lib_update_H(fake, fake, fake, 8, 8, 2, None, ws, 1 << 30, null, null, null, null) == 1
    msg = dna._lib_last_error().decode()
    assert "opts" in msg
    # eq. (2) weights: finite and >= 0
    for kw in ({"rho": -0.5}, {"lam": -1e-3}, {"rho": float("nan")}, {"lam": float("inf")}):
        bad = dna.make_opts(**kw)
        assert E(fake, fake, fake, 8, 8, 2, ctypes.byref(bad), ws, 1 << 30, null, null, null, null) == 1, kw
        assert "rho and lambda" in dna._lib_last_error().decode()
    # the unrolled adjoint has no lambda terms
    reg = dna.make_opts(lam=0.5)
    assert dna._lib_ufwd(fake, fake, fake, 2, 8, 8, 2, ctypes.byref(reg), fake, fake, ws, 1 << 30, null) == 6
    assert dna._lib_ubwd(fake, fake, fake, fake, 2, 8, 8, 2, fake, fake, fake, null, ctypes.byref(reg), ws,
                         1 << 30, null) == 6
    # side out of range, with_cost without output
    assert dna._lib_normalize(2, fake, fake, 8, 8, 2, ctypes.byref(o), ws, 1 << 30, null) == 1
    assert dna._lib_mu(0, fake, fake, fake, 8, 8, 2, 1, null, ctypes.byref(o), ws, 1 << 30, null) == 1
    assert dna._lib_kl(fake, fake, fake, 8, 8, 2, ctypes.byref(o), ws, 1 << 30, null, null) == 1
    # whole iterations: null factor, negative count, small workspace; zero iterations enqueue nothing
    It = dna._lib_iterate
    assert It(fake, fake, null, 8, 8, 2, 3, ctypes.byref(o), ws, 1 << 30, null) == 1
    assert It(fake, fake, fake, 8, 8, 2, -1, ctypes.byref(o), ws, 1 << 30, null) == 1
    assert It(fake, fake, fake, 8, 8, 2, 3, ctypes.byref(o), ws, 16, null) == 2
    assert It(fake, fake, fake, 8, 8, 2, 0, ctypes.byref(o), ws, 1 << 30, null) == 0
    Mi = dna._lib_mu_it
    assert Mi(fake, null, fake, 8, 8, 2, 3, 0, ctypes.byref(o), ws, 1 << 30, null) == 1
    assert Mi(fake, fake, fake, 8, 8, 2, -2, 0, ctypes.byref(o), ws, 1 << 30, null) == 1
    assert Mi(fake, fake, fake, 8, 8, 2, 0, 1, ctypes.byref(o), ws, 1 << 30, null) == 0


def test_build_info_names_target():
    from paper_1301_3389_amd import dna
    assert "gfx950" in dna.build_info()
