"""Host-side checks of the C ABI library (no GPU needed): it loads and exports every symbol that
include/lind.h declares, and the header and the binding agree on the struct layouts."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lind.h")
LIB = os.path.join(ROOT, "paper_2608_30860_amd", "liblindx.so")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lind_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2608_30860_amd.build import build
        build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert "lind_create" in names and "lind_steady_state" in names
    for name in names:
        assert hasattr(lib, name), name


def test_every_internal_symbol_is_exported(lib):
    """include/lind_internal.h (kernel-level entry points for the tests and the benchmark): every
    declared function is exported by the library."""
    txt = open(os.path.join(ROOT, "include", "lind_internal.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = sorted(set(re.findall(r"\b(lindx_[a-z0-9_]+)\s*\(", txt)))
    assert "lindx_trisylv_blk" in names and "lindx_p4_test" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_symbol_list_matches_header():
    from paper_2608_30860_amd import SYMBOLS
    assert sorted(SYMBOLS) == header_functions()


def test_default_opts_and_struct_layout(lib):
    from paper_2608_30860_amd.lindx import LindInfo, LindOpts
    o = LindOpts()
    lib.lind_default_opts(ctypes.byref(o))
    assert (o.prec, o.route, o.m, o.max_restarts, o.refine_max) == (0, 0, 30, 200, 8)
    assert o.kappa_max == 1e3 and o.eta == 1.0 and o.stream is None
    # compare every field offset with the C compiler's layout of include/lind.h
    import subprocess
    import tempfile
    fields = [("lind_opts", LindOpts), ("lind_info", LindInfo)]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "lind.h"', "int main(void){"]
    for cname, cls in fields:
        src.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            src.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    src.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        open(c, "w").write("\n".join(src))
        exe = os.path.join(d, "layout")
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        got = [int(x) for x in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    want = []
    for _, cls in fields:
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f).offset for f, _ in cls._fields_]
    assert got == want


def test_create_rejects_bad_arguments_without_touching_a_device(lib):
    h = ctypes.c_void_p()
    lib.lind_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                ctypes.c_int, ctypes.c_void_p]
    assert lib.lind_create(ctypes.byref(h), None, None, 4, 1, None) == -1   # NULL H
    assert lib.lind_create(ctypes.byref(h), ctypes.c_void_p(16), None, 0, 0, None) == -1  # n < 1
    assert lib.lind_create(None, ctypes.c_void_p(16), None, 4, 0, None) == -1
    lib.lind_last_error.restype = ctypes.c_char_p
    assert b"invalid" in lib.lind_last_error(None) or b"NULL" in lib.lind_last_error(None)
    assert lib.lind_create(ctypes.byref(h), ctypes.c_void_p(16), None, 10241, 0, None) == -1  # n > LIND_NMAX
    assert b"10240" in lib.lind_last_error(None)


def test_triangular_solves_check_sizes_without_touching_a_device(lib):
    """n = 0 is an empty solve; a negative n, or one whose column does not fit in LDS, is refused
    before any workspace is allocated or kernel launched."""
    for name in ("lindx_trevec", "lindx_triinv"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        assert f(None, None, 0, None) == 0
        assert f(None, None, -3, None) == -1
        assert f(None, None, 10241, None) == -1


def test_binding_rejects_host_tensors_and_wrong_dtypes():
    """The Python binding hands the library device pointers only: host tensors and other dtypes
    are refused before lind_create is called (so no device is touched)."""
    torch = pytest.importorskip("torch")
    from paper_2608_30860_amd import Lindblad
    H = torch.zeros((4, 4), dtype=torch.complex128)
    Ls = torch.zeros((1, 4, 4), dtype=torch.complex128)
    with pytest.raises(TypeError, match="CUDA"):
        Lindblad(H, Ls)
    with pytest.raises(TypeError, match="complex128"):
        Lindblad(H.to(torch.complex64), Ls)


def test_small_product_ksplit_plan(lib):
    """The K-split plan of single small products (host logic, no GPU): the chunk count divides K,
    every chunk is at least 32 deep, the partials fit the workspace, the split workgroups stay
    within one round of 256 compute units, and large products or a missing workspace are not
    split.  Concrete cases: the basis change of n = 256 (64 tiles of 32 x 32, four chunks), the
    stacked product of the dephased Kerr cavity at n = 512 in FP64 (128 tiles of 64 x 64, two)."""
    f = lib.lindx_gemm_ksplit
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_longlong]
    f.restype = ctypes.c_int
    big = 1 << 40
    assert f(0, 256, 256, 256, big) == 4
    assert f(1, 256, 256, 256, big) == 4
    assert f(0, 1024, 512, 512, big) == 2
    assert f(0, 512, 256, 256, big) == 2
    assert f(0, 96, 80, 250, big) == 2
    assert f(0, 37, 45, 29, big) == 1
    assert f(0, 2048, 2048, 2048, big) == 1
    assert f(1, 2048, 2048, 2048, big) == 1
    assert f(2, 256, 256, 256, big) == 1  # BF16x3 products are not split this way
    assert f(0, 256, 256, 256, 0) == 1
    assert f(0, 256, 256, 256, 2 * 256 * 256 * 16) == 2  # workspace for two partials only
    assert f(3, 256, 256, 256, big) == -1

    def tiles(M, N, b):
        return ((M + b - 1) // b) * ((N + b - 1) // b)

    rng = np.random.default_rng(0)
    for _ in range(400):
        M, N, K = (int(v) for v in rng.integers(1, 1300, size=3))
        prec = int(rng.integers(0, 2))
        ws = int(rng.choice([0, 1 << 20, 1 << 26, big]))
        ks = f(prec, M, N, K, ws)
        assert ks in (1, 2, 4, 8), (prec, M, N, K, ws, ks)
        if ks == 1:
            continue
        elem = 16 if prec == 0 else 8
        assert K % ks == 0 and K // ks >= 32
        assert ks * M * N * elem <= ws
        if prec == 0:
            bt = 64 if tiles(M, N, 64) >= 128 else 32
        else:
            bt = 32
        assert tiles(M, N, bt) * ks <= 256
        assert tiles(M, N, 128) < 96


def test_p4_split_run_count(lib):
    """The split-K run count of the pre-split BF16 product (host logic, no GPU): within [1, 64] and
    never more runs than 32-deep stages; one run when the tiles alone fill whole rounds of the
    chip; the jump reduction of the n = 2048, d = 8 workload (136 upper tiles, 8 products of 2048)
    in 9 runs, so that its 1224 workgroups fill whole rounds of 256 compute units but the last."""
    f = lib.lindx_p4_pick_split
    f.argtypes = [ctypes.c_longlong, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    f.restype = ctypes.c_int
    assert f(136, 8, 2048, 256) == 9
    assert f(2048, 1, 2048, 256) == 1
    assert f(256, 1, 2048, 256) == 1
    assert f(1, 1, 1, 256) == 1
    assert f(-1, 1, 1, 256) == -1
    rng = np.random.default_rng(1)
    for _ in range(300):
        tiles = int(rng.integers(1, 3000))
        nb = int(rng.integers(1, 12))
        k = int(rng.integers(1, 5000))
        cus = int(rng.choice([64, 256, 304]))
        s = f(tiles, nb, k, cus)
        stages = nb * ((k + 31) // 32)
        assert 1 <= s <= min(64, stages), (tiles, nb, k, cus, s)
        if tiles % cus == 0:
            assert s == 1  # whole rounds already: splitting only adds partial-sum traffic
