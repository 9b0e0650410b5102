"""Host-only checks of the C ABI: the library loads, exports every function
the header declares, the ctypes structure matches the C layout, and the
library's flop model agrees with the oracle's.  No GPU compute is called."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2508_19138_amd import qtx_rgf as Q
from oracle.flops import rgf_flops, w_assembly_flops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtx_rgf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qtx_rgf_\w+)\s*\(", src)))


def test_header_declares_core_entry_points():
    names = _declared()
    for n in ("qtx_rgf_create", "qtx_rgf_solve_batch", "qtx_rgf_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = Q.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(Q.exported_symbols()) == _declared()


@pytest.mark.parametrize("cname,pystruct", [("qtx_rgf_problem", "Problem"),
                                             ("qtx_rgf_completion", "Completion"),
                                             ("qtx_rgf_nested", "Nested")])
def test_struct_layout_matches_c(tmp_path, cname, pystruct):
    """Compile a tiny C program against the header (gcc, host only) and
    compare sizeof/offsetof with the ctypes mirror."""
    S = getattr(Q, pystruct)
    fields = [f[0] for f in S._fields_]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "qtx_rgf.h"',
            "int main(void){", 'printf("%%zu\\n", sizeof(%s));' % cname]
    for f in fields:
        prog.append('printf("%%zu\\n", offsetof(%s, %s));' % (cname, f))
    prog.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(S)
    for f, off in zip(fields, out[1:]):
        assert int(off) == getattr(S, f).offset, f


@pytest.mark.parametrize("n,b", [(1, 8), (2, 32), (8, 32), (32, 512), (17, 100)])
def test_flop_model_matches_oracle(n, b):
    for bt in (False, True):
        assert Q.flops_per_energy(Q.QTX_KIND_G, n, b, 2, bt) == rgf_flops(n, b, 2, bt)
        assert Q.flops_per_energy(Q.QTX_KIND_G, n, b, 1, bt) == rgf_flops(n, b, 1, bt)
    w = Q.flops_per_energy(Q.QTX_KIND_W, n, b, 2, True, True)
    assert w == rgf_flops(n, b, 2, True) + w_assembly_flops(n, b, 2, True)


def test_status_strings():
    for st in range(8):
        assert Q.status_string(st)


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    st = Q.lib().qtx_rgf_create(ctypes.byref(h), 0, 0, None, 0)
    assert st != Q.QTX_OK and not h.value
    st = Q.lib().qtx_rgf_create(ctypes.byref(h), -1, 0, None, 0)
    assert st == Q.QTX_ERR_INVALID_ARG


def test_occupation_arrays_are_checked_before_the_call():
    """The lesser/greater binding refuses host occupation arrays shorter than
    the batch before reaching the library (no device needed)."""
    import numpy as np
    from paper_2508_19138_amd import qtx_rgf as Q
    ctx = Q.Context.__new__(Q.Context)            # no device: the check comes first
    with pytest.raises(ValueError):
        Q.Context.obc_lesser_greater(ctx, 4, 3, None, 0, np.ones(2), np.ones(3), None, None)


def test_noalloc_scratch_size_matches_header():
    src = open(HEADER).read()
    m = re.search(r"#define QTX_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", src)
    assert m, "QTX_NOALLOC_SCRATCH_BYTES not found"
    assert Q.QTX_NOALLOC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))


def test_panel_kernel_rows_stay_in_registers(tmp_path):
    """The inverse's panel kernel holds R rows of the panel per thread in
    registers; compiled with the library's options (hipcc cross-compiles
    for gfx950 without a device), the instances for R = 1..3 must not place
    that array in scratch memory (nor the tall path's chunk and final
    instances, nor the one-workgroup inverse its tile)."""
    from paper_2508_19138_amd import build as B
    src = os.path.join(B.CSRC, "zinv.hip")
    out = str(tmp_path / "zinv.s")
    cmd = ([B.HIPCC] + B.COMMON + B.PER_FILE["zinv.hip"] +
           ["-x", "hip", "-S", "--cuda-device-only", src, "-o", out])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    meta = open(out).read()
    # (R, mode): whole-matrix panels, and the tall path's chunk and final steps
    for R, mode in ((1, 0), (2, 0), (3, 0), (3, 1), (1, 2)):
        name = "_ZN3qtx12_GLOBAL__N_115gj_panel_kernelILi%dELi%dEEEvNS_10FlatLaunchEi" % (R, mode)
        # the kernel's entry in the code-object metadata
        i = meta.index(".name:           " + name)
        lo = meta.rindex("\n  - .", 0, i)
        hi = meta.find("\n  - .", i)
        block = meta[lo:hi if hi >= 0 else len(meta)]
        m = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
        assert m and int(m.group(1)) == 0, (R, mode, m and m.group(1))
    # the one-workgroup inverse: its tile of TR x 4 complex entries per lane
    # (256 or 512 bytes) stays in registers; a few spilled words of the
    # set-up are allowed
    for TR in (4, 8):
        name = "_ZN3qtx12_GLOBAL__N_115gj_small_kernelILi%dEEEvNS_10FlatLaunchE" % TR
        i = meta.index(".name:           " + name)
        lo = meta.rindex("\n  - .", 0, i)
        hi = meta.find("\n  - .", i)
        block = meta[lo:hi if hi >= 0 else len(meta)]
        m = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
        assert m and int(m.group(1)) <= 32, (TR, m and m.group(1))
