"""Host-side checks of the C ABI library (no GPU): it is built for gfx950,
loads, and exports every function include/dda.h declares with the ctypes
signatures the binding uses; struct layouts match the header."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dda.h")
LIB = os.path.join(ROOT, "paper_1202_3424_amd", "libdda.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dda_[a-z_]+)\s*\(", src)))


def _lib():
    if not os.path.exists(LIB):
        from paper_1202_3424_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("dda_ctx_create", "dda_ctx_destroy", "dda_target_create", "dda_target_destroy", "dda_solve",
              "dda_solve_batched", "dda_grad_eps", "dda_apply", "dda_last_error", "dda_target_geometry"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_covers_every_declared_symbol():
    from paper_1202_3424_amd import _abi
    assert sorted(_abi.SIGNATURES) == _declared()


def test_struct_sizes_match_header():
    """Compile a tiny C program against the header and compare sizeof()."""
    from paper_1202_3424_amd import _abi
    prog = ('#include "dda.h"\n#include <stdio.h>\n'
            'int main(){printf("%zu %zu %zu %zu\\n", sizeof(dda_c64), sizeof(dda_incidence), sizeof(dda_opts),'
            ' sizeof(dda_result));return 0;}\n')
    tmp = os.path.join(ROOT, "_build")
    os.makedirs(tmp, exist_ok=True)
    c = os.path.join(tmp, "sizes.c")
    exe = os.path.join(tmp, "sizes")
    open(c, "w").write(prog)
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
    sizes = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert sizes == [ctypes.sizeof(_abi.C64), ctypes.sizeof(_abi.Incidence), ctypes.sizeof(_abi.Opts),
                     ctypes.sizeof(_abi.Result)]


def test_last_error_is_callable_without_gpu():
    lib = _lib()
    lib.dda_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.dda_last_error(), bytes)


def test_library_targets_gfx950():
    """The offload bundle inside the library carries a gfx950 code object."""
    sec = os.path.join(ROOT, "_build", "fatbin.bin")
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", LIB, sec], check=True)
    data = open(sec, "rb").read()
    assert b"gfx950" in data
