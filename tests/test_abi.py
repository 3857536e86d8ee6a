"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and its host-side validation and footprint logic behave."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fctn.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(fctn_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def F():
    from paper_2510_22506_amd import fctn
    if not os.path.exists(fctn.LIB_PATH):
        pytest.fail("libfctn.so is not built (run __graft_entry__.build())")
    fctn.lib()
    return fctn


def test_exports_every_declared_symbol(F):
    names = _declared()
    assert len(names) >= 18
    raw = ctypes.CDLL(F.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n


def test_status_strings(F):
    for s in range(7):
        assert F.fctn_status_str(s) and F.fctn_status_str(s) != 'unknown status'


def test_workspace_bytes_and_validation(F):
    d = F.make_desc((32, 32, 8), (3, 3, 3), precision="f64")
    n = F.fctn_workspace_bytes(d)
    assert n > 32 * 32 * 8 * 8 * 2 and n % 256 == 0
    # invalid descriptors give 0
    bad = [F.make_desc((32, 0, 8), (3, 3, 3)), F.make_desc((32, 32, 8), (3, 0, 3)),
           F.make_desc((32, 32, 8), (3, 3, 3), rho=0.0),
           F.make_desc((32, 32, 8), (3, 3, 3), lam=-1.0),
           F.make_desc((32, 32, 8), (3, 3, 3), extrapolation=(1.0, 0.5)),
           F.make_desc((32, 32, 8), (3, 3, 3), extrapolation=(-0.1, 0.5)),
           F.make_desc((32, 32, 8), (3, 3, 3), extrapolation=(0.5, 1.5))]
    for b in bad:
        assert F.fctn_workspace_bytes(b) == 0
    assert F.fctn_workspace_bytes(F.make_desc((32, 32, 8), (3, 3, 3), precision="f64",
                                              extrapolation=(0.5, 0.5))) == n
    # orders up to 8 plan when their rank products fit the solve
    assert F.fctn_workspace_bytes(F.make_desc((3,) * 7, (2,) * 21)) > 0
    r8 = (1, 2, 1, 2, 2, 1, 1, 2, 1, 2, 1, 1, 2, 2, 1, 2, 1, 1, 2, 1, 2, 2, 1, 1, 2, 1, 2, 1)
    assert F.fctn_workspace_bytes(F.make_desc((2, 3, 2, 2, 3, 2, 2, 3), r8)) > 0
    # valid for the method, outside the library's support: N = 2, rank
    # products above 192 (3^6 at every mode of this order 7 tensor), and an
    # order 8 tensor whose middle modes have 2^16 cross bonds between the two
    # operand runs (a slab of them does not fit in LDS)
    assert F.fctn_workspace_bytes(F.make_desc((3,) * 7, (3,) * 21)) == 0
    assert F.fctn_workspace_bytes(F.make_desc((3,) * 8, (2,) * 28)) == 0
    assert F.fctn_workspace_bytes(F.make_desc((5, 4), (2,))) == 0
    assert F.fctn_workspace_bytes(F.make_desc((8, 8, 8), (16, 16, 2))) == 0


def test_footprint_scales_with_tensor(F):
    a = F.fctn_workspace_bytes(F.make_desc((144, 176, 3, 50), (8, 3, 8, 3, 8, 3)))
    b = F.fctn_workspace_bytes(F.make_desc((144, 176, 3, 25), (8, 3, 8, 3, 8, 3)))
    assert a > b > 0
    # X and Z (float32) plus the larger pair tensor are at least this much
    assert a >= 2 * 4 * 144 * 176 * 3 * 50 + 4 * 144 * 176 * 576


def test_mode_sizes(F):
    d = F.make_desc((144, 176, 3, 50), (8, 3, 8, 3, 8, 3))
    assert [F.fctn_mode_sizes(d, k) for k in range(4)] == [(192, 144), (192, 176), (27, 3), (192, 50)]
    with pytest.raises(F.FctnError):
        F.fctn_mode_sizes(d, 4)
    d5 = F.make_desc((6, 5, 4, 3, 2), (2, 3, 1, 2, 3, 1, 2, 2, 1, 3))
    # s_k = product of the bonds at k, e.g. s_1 = R12 R13 R14 R15 = 2 * 3 * 1 * 2
    assert [F.fctn_mode_sizes(d5, k) for k in range(5)] == \
        [(12, 6), (12, 5), (18, 4), (6, 3), (12, 2)]


def test_plan_rejects_bad_arguments_without_touching_the_device(F):
    d = F.make_desc((8, 8, 8), (2, 2, 2))
    h = ctypes.c_void_p()
    lib = F.lib()
    # null workspace and misaligned workspace are rejected before any HIP call
    assert lib.fctn_plan(ctypes.byref(d), None, 1 << 20, None, None, 0,
                         ctypes.byref(h)) == F.E_INVALID
    assert lib.fctn_plan(ctypes.byref(d), ctypes.c_void_p(16), 1 << 20, None, None, 0,
                         ctypes.byref(h)) == F.E_INVALID
    assert lib.fctn_plan(ctypes.byref(d), ctypes.c_void_p(4096), 16, None, None, 0,
                         ctypes.byref(h)) == F.E_NOMEM
    assert lib.fctn_sweep(None, 1, None) == F.E_INVALID
    assert lib.fctn_destroy(None) == F.E_INVALID


def test_every_small_shape_is_supported(F):
    import itertools
    bad = []
    for dims in itertools.product([1, 2, 3, 5, 7, 16, 33], [1, 3, 4, 17], [1, 2, 3, 5]):
        for p in ("f64", "f32"):
            if F.fctn_workspace_bytes(F.make_desc(dims, (2, 3, 2), precision=p)) == 0:
                bad.append((dims, p))
    for dims in [(1, 1, 1, 1), (2, 3, 1, 2), (13, 11, 3, 7), (5, 3, 3, 2)]:
        if F.fctn_workspace_bytes(F.make_desc(dims, (2,) * 6, precision="f32")) == 0:
            bad.append(dims)
    # orders 5 and 6 (operand groups built per mode)
    for dims in [(1, 1, 1, 1, 1), (3, 4, 2, 5, 3), (9, 7, 3, 4, 5), (2, 3, 2, 2, 3, 2)]:
        ranks = (2,) * (len(dims) * (len(dims) - 1) // 2)
        for p in ("f64", "f32", "bf16x3"):
            if F.fctn_workspace_bytes(F.make_desc(dims, ranks, precision=p)) == 0:
                bad.append((dims, p))
    assert not bad


def test_struct_layouts_match_header(F, tmp_path):
    # the ctypes mirrors of the C structs have the size and field offsets a C
    # compiler gives the header's declarations
    structs = {"fctn_desc": F.fctn_desc, "fctn_sweep_stats": F.fctn_sweep_stats,
               "fctn_stats": F.fctn_stats, "fctn_request": F.fctn_request,
               "fctn_completion": F.fctn_completion}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fctn.h"',
             'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for fld, _ in cls._fields_:
            cf = "lambda" if fld == "lambda_" else fld
            lines.append(f'  printf("{name}.{fld} %zu\\n", offsetof({name}, {cf}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fld, _ in cls._fields_:
            assert int(got[f"{name}.{fld}"]) == getattr(cls, fld).offset, (name, fld)
