"""C-interface checks that need no GPU: the library loads, exports every
function declared in include/proxsdp.h, and the host-only entry points
(validation, workspace sizing) behave as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1810_05231_amd import _lib
    return _lib


def test_exports_every_declared_symbol():
    L = _lib()
    header = open(os.path.join(ROOT, "include", "proxsdp.h")).read()
    names = set(re.findall(r"\b(proxsdp_[a-z_]+)\s*\(", header))
    assert {"proxsdp_create", "proxsdp_step", "proxsdp_solve", "proxsdp_project_psd"} <= names
    for name in sorted(names):
        assert hasattr(L.lib, name), name


def test_struct_layouts_match_header(tmp_path):
    """Field offsets of the ctypes mirrors equal those gcc computes from the header."""
    import shutil
    import subprocess
    L = _lib()
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"proxsdp_problem": L.Problem, "proxsdp_options": L.Options, "proxsdp_info": L.Info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "proxsdp.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_default_options():
    L = _lib()
    o = L.default_options()
    assert o.tol == 1e-4 and o.window == 50 and o.check_every == 10 and o.r0 == 1
    assert o.precision == L.FP64 and o.row_scaling == 1


def _size(prob, **opt):
    from paper_1810_05231_amd import workspace_size
    return workspace_size(prob, **opt)


def test_workspace_size_grows_with_n():
    s1 = _size(I.maxcut(100, 0.1, 0))
    s2 = _size(I.maxcut(400, 0.1, 0))
    s3 = _size(I.maxcut(1600, 0.02, 0))
    assert 0 < s1 < s2 < s3
    # the dense n x n iterate dominates: at least 8 n^2 bytes
    assert s3 >= 8 * 1600 * 1600


def _expect_error(code, prob, **opt):
    from paper_1810_05231_amd import ProxSDPError
    with pytest.raises(ProxSDPError) as ei:
        _size(prob, **opt)
    assert ei.value.code == code
    return str(ei.value)


def test_rejects_lower_triangle_entries():
    L = _lib()
    p = I.maxcut(10, 0.5, 0)
    p.c_i, p.c_j = p.c_j.copy(), p.c_i.copy()    # swap to the lower triangle
    msg = _expect_error(L.PROXSDP_ERR_INVALID, p)
    assert "below the diagonal" in msg


def test_rejects_out_of_range_and_nonfinite():
    L = _lib()
    p = I.maxcut(10, 0.5, 0)
    p.a_j = p.a_j.copy()
    p.a_j[0] = 10
    _expect_error(L.PROXSDP_ERR_INVALID, p)
    p = I.maxcut(10, 0.5, 0)
    p.c_v = p.c_v.copy()
    p.c_v[0] = np.nan
    _expect_error(L.PROXSDP_ERR_INVALID, p)
    p = I.maxcut(10, 0.5, 0)
    p.a_row = p.a_row.copy()
    p.a_row[0] = p.m + p.p
    _expect_error(L.PROXSDP_ERR_INVALID, p)


def test_rejects_zero_row_and_bad_options():
    L = _lib()
    p = I.maxcut(10, 0.5, 0)
    p.a_v = p.a_v.copy()
    p.a_v[3] = 0.0
    assert "is zero" in _expect_error(L.PROXSDP_ERR_INVALID, p)
    p = I.maxcut(10, 0.5, 0)
    _expect_error(L.PROXSDP_ERR_INVALID, p, window=45, check_every=10)
    _expect_error(L.PROXSDP_ERR_INVALID, p, tol=0.0)
    _expect_error(L.PROXSDP_ERR_UNSUPPORTED, I.maxcut(100, 0.1, 0), full_eig=1)
    _expect_error(L.PROXSDP_ERR_INVALID, p, block=24)
    _expect_error(L.PROXSDP_ERR_INVALID, p, rank_test=2)
    _expect_error(L.PROXSDP_ERR_INVALID, p, block=-16)


def test_fixed_block_caps_the_rank():
    # a fixed subspace width k caps r at k (k - 1 with the lambda_{r+1} test):
    # the workspace of block=16 does not grow with r0 or r_max (the factor
    # and basis blocks are sized by the width), so r can never exceed k
    L = _lib()
    p = I.maxcut(300, 0.05, 0)
    s16 = _size(p, block=16)
    assert _size(p, block=16, r0=40, r_max=60) == s16
    assert _size(p, block=16, rank_test=L.RANK_TEST_LAMBDA_R_PLUS_1) == s16
    assert _size(p, r0=40) > s16


def test_default_rank_test_is_lambda_r():
    L = _lib()
    assert L.default_options().rank_test == L.RANK_TEST_LAMBDA_R


def test_project_workspace_size_limits():
    L = _lib()
    nb = C.c_size_t()
    assert L.lib.proxsdp_project_workspace_size(50, 0, L.FP64, C.byref(nb)) == 0
    assert nb.value > 0
    assert L.lib.proxsdp_project_workspace_size(1000, 8, L.FP64, C.byref(nb)) == 0
    # exact projection beyond the single-workgroup eigensolver size goes
    # through rocSOLVER, whose scratch size needs a device (HIP error here
    # without one); a partial rank above the cap is unsupported
    assert L.lib.proxsdp_project_workspace_size(1000, 0, L.FP64, C.byref(nb)) in (0, L.PROXSDP_ERR_HIP)
    assert L.lib.proxsdp_project_workspace_size(1000, 100, L.FP64, C.byref(nb)) == L.PROXSDP_ERR_UNSUPPORTED
    assert L.lib.proxsdp_project_workspace_size(0, 1, L.FP64, C.byref(nb)) == L.PROXSDP_ERR_INVALID


def test_duplicates_are_summed_in_sizing():
    # duplicated triplets are accepted (summed), same workspace as the merged problem
    p = I.maxcut(20, 0.3, 1)
    q = I.maxcut(20, 0.3, 1)
    q.c_i = np.concatenate([q.c_i, q.c_i[:5]])
    q.c_j = np.concatenate([q.c_j, q.c_j[:5]])
    q.c_v = np.concatenate([q.c_v * 0.5, q.c_v[:5] * 0.0])
    assert _size(p) == _size(q)
