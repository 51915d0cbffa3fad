"""CPU-only checks of the C-ABI library: it loads, exports every declared entry point,
reports its defaults, and rejects malformed inputs during host-side validation (before any
device call, so these run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1507_08157_amd import binding
from synth import abi as sabi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "tddft.h")).read()
    return sorted(set(re.findall(r"\b(tddft_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    names = _declared()
    assert "tddft_apply" in names and "tddft_pcg_solve" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(binding.EXPORTS) == set(names)


def test_abi_version_and_strings():
    assert binding.tddft_abi_version() == 1
    assert binding.tddft_strerror(binding.TDDFT_E_NOT_PD) == "not positive definite"
    assert binding.tddft_strerror(12345) == "unknown status"


def test_default_options():
    o = binding.tddft_default_options()
    assert o.precision == binding.TDDFT_FP64
    assert o.precond == binding.TDDFT_PC_KSDIFF_CG
    assert o.eps_tol == 1e-4 and o.tol_omega == 1e-7 and o.max_iter == 300
    assert o.rho_floor == 1e-10 and o.coupling_scale == 1.0 and o.refresh == 10
    assert o.density_pbcast == -1 and o.gemm_tile == -1
    assert o.sparse_cw == -1 and o.sparse_pairs == -1


def _c_layout(struct, fields):
    """sizeof and offsetof of a header struct, from a C program built with gcc."""
    import subprocess
    import tempfile
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tddft.h"', 'int main(void){',
             f'printf("%zu\\n", sizeof({struct}));']
    lines += [f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines.append('return 0;}')
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    return [int(x) for x in out]


@pytest.mark.parametrize("cls", ["tddft_bsr", "tddft_functions", "tddft_system",
                                 "tddft_options", "tddft_stats", "tddft_info"])
def test_binding_struct_layout_matches_header(cls):
    st = getattr(binding, cls)
    names = [f[0] for f in st._fields_]
    c = _c_layout(cls, names)
    assert c[0] == C.sizeof(st)
    for name, off in zip(names, c[1:]):
        assert getattr(st, name).offset == off, name


@pytest.fixture(scope="module")
def arrays(small_odd):
    return sabi.system_arrays(small_odd)


def _expect_invalid(arrays, match):
    with pytest.raises(binding.TddftError) as e:
        binding.tddft_create(arrays)
    assert e.value.code == binding.TDDFT_E_INVALID
    assert match in str(e.value)


def _copy(a):
    import copy
    return copy.deepcopy(a)


def test_rejects_grid_not_2357(arrays):
    a = _copy(arrays)
    a["n"] = np.array([44, 45, 45], dtype=np.int32)   # 44 = 4 * 11
    _expect_invalid(a, "products of 2, 3, 5 and 7")


def test_rejects_asymmetric_overlap(arrays):
    a = _copy(arrays)
    a["S_u"]["val"] = a["S_u"]["val"].copy()
    a["S_u"]["val"][1] += 1e-3
    _expect_invalid(a, "S_u: matrix not symmetric")


def test_rejects_nan(arrays):
    a = _copy(arrays)
    a["H_o"]["val"] = a["H_o"]["val"].copy()
    a["H_o"]["val"][0] = np.nan
    _expect_invalid(a, "non-finite")


def test_rejects_unsorted_pattern(arrays):
    a = _copy(arrays)
    ci = a["M"]["colind"].copy()
    if a["M"]["rowptr"][1] >= 2:
        ci[0], ci[1] = ci[1], ci[0]
    a["M"]["colind"] = ci
    _expect_invalid(a, "M: columns not strictly increasing")


def test_rejects_box_larger_than_cell(arrays):
    a = _copy(arrays)
    ext = a["vir"]["extent"].copy()
    ext[0] = 1000
    a["vir"]["extent"] = ext
    _expect_invalid(a, "box larger than the cell")


def test_rejects_block_size(arrays):
    a = _copy(arrays)
    # one o-block of 6 functions
    off = a["S_o"]["row_off"].copy()
    off[1:] = off[1:] + 4
    off[-1] = a["S_o"]["row_off"][-1]
    a["S_o"]["row_off"] = off
    _expect_invalid(a, "block sizes must be 1..5")


def test_joint_blocks_pass_the_host_checks():
    """5 u-functions x 2 o-functions per atom (the joint representation) select the 5 x 2
    padded shape: every host-side step, which copies each block into its padded one, runs
    to the first device call (on a machine without a GPU that call fails cleanly)."""
    from conftest import cached_system
    s = cached_system("small_joint")
    try:
        h = binding.tddft_create(sabi.system_arrays(s), precision="fp64")
    except binding.TddftError as e:
        assert e.code == binding.TDDFT_E_DEVICE, str(e)
        return
    info = h.tddft_get_info()
    h.close()
    assert (info["block_rows"], info["block_cols"]) == (5, 2)


def test_rejects_uncovered_block_shape(arrays):
    """5 u-functions with 3 o-functions per atom fit no padded shape."""
    a = _copy(arrays)
    for name in ("S_o", "H_o", "K_v"):
        off = a[name]["row_off"].copy()
        off[1:] = off[1:] + 1                 # first o-block: 3 functions
        off[-1] = a[name]["row_off"][-1]
        a[name]["row_off"] = off
    uoff = a["S_u"]["row_off"].copy()
    uoff[1:] = uoff[1:] + 2                   # first u-block: 5 functions
    uoff[-1] = a["S_u"]["row_off"][-1]
    a["S_u"]["row_off"] = uoff
    with pytest.raises(binding.TddftError) as e:
        binding.tddft_create(a)
    assert e.value.code == binding.TDDFT_E_INVALID


@pytest.mark.parametrize("cw,pb", [(3, 1), (1, -1), (-1, 4), (4, 4), (2, 8), (1, 3)])
def test_rejects_unknown_sparse_variant(arrays, cw, pb):
    """Forced sparse-product variants must be one of the built (columns, pairs) forms; the
    check runs before any device call."""
    with pytest.raises(binding.TddftError) as e:
        binding.tddft_create(arrays, sparse_cw=cw, sparse_pairs=pb)
    assert e.value.code == binding.TDDFT_E_INVALID and "sparse_cw" in str(e.value)
