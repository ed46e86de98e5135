"""C ABI checks that need no GPU: the library loads, exports every function
include/ecg.h declares, and rejects invalid arguments before touching a
device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1804_10629_amd as E
import problems as P
from tests.conftest import ROOT, gpu_available

HEADER = os.path.join(ROOT, "include", "ecg.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ecg_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(E.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert set(names) <= set(E._SIGS)


def test_version_and_strings():
    assert "gfx950" in E.version()
    for code in (0, 1, 2, 3, -1, -2, -3, -4):
        assert E.strerror(code) and E.strerror(code) != "unknown status"
    assert E.strerror(99) == "unknown status"
    assert [E.lib.ecg_kclass_name(i).decode() for i in range(10)] == E.KCLASSES
    assert E.lib.ecg_kclass_name(10) is None


def test_opts_default():
    o = E._Opts()
    E.lib.ecg_opts_default(ctypes.byref(o))
    assert (o.variant, o.orth, o.precision, o.device_ptrs) == (0, 0, 0, 0)
    assert o.inner_tol == 1e-4 and o.max_restarts == 20 and o.grid == 0
    assert list(o.reserved) == [0]
    assert o.ca == 0 and o.row_key is None
    assert o.permute_domains == 1 and o.progress_every == 0


def _setup(n, rowptr, colind, vals, part, t, s, **kw):
    o = E._Opts()
    E.lib.ecg_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    ctx = ctypes.c_void_p()
    args = [np.ascontiguousarray(a) for a in (rowptr, colind, vals, part)]
    code = E.lib.ecg_setup(ctypes.byref(ctx), n, *(a.ctypes.data for a in args), t, s,
                           ctypes.byref(o))
    if ctx.value:
        E.lib.ecg_destroy(ctx)
    return code, E.lib.ecg_last_error().decode()


@pytest.fixture(scope="module")
def small():
    p = P.poisson2d(8, t=4, parts=(2, 2, 1))
    dom = np.repeat(np.arange(4, dtype=np.int32), 16)
    return p, dom


@pytest.mark.parametrize("case", [
    "n0", "t0", "t65", "t_gt_n", "s0", "s17", "rowptr0", "decreasing", "col_range",
    "part_range", "empty_domain", "nan_value", "reserved", "variant", "inner_tol", "q_cap",
    "ca", "row_key"])
def test_setup_rejects(small, case):
    p, dom = small
    rp, ci, va, pd = p.rowptr.copy(), p.colind.copy(), p.vals.copy(), dom.copy()
    n, t, s, kw = p.n, 4, 2, {}
    if case == "n0":
        n = 0
    elif case == "t0":
        t = 0
    elif case == "t65":
        t = 65
    elif case == "t_gt_n":
        n, t = 3, 4
        rp = rp[:4]
    elif case == "s0":
        s = 0
    elif case == "s17":
        s = 17
    elif case == "rowptr0":
        rp = rp + 1
    elif case == "decreasing":
        rp[5] = rp[7]
    elif case == "col_range":
        ci[3] = p.n
    elif case == "part_range":
        pd[0] = 4
    elif case == "empty_domain":
        pd[pd == 2] = 1
    elif case == "nan_value":
        va[10] = np.nan
    elif case == "reserved":
        kw = {"reserved": (ctypes.c_int32 * 1)(1)}
    elif case == "variant":
        kw = {"variant": 7}
    elif case == "inner_tol":
        kw = {"inner_tol": 1.5}
    elif case == "q_cap":
        kw = {"variant": E.SRECG2, "q_cap_blocks": 1}
    elif case == "ca":
        kw = {"ca": 3}
    elif case == "row_key":   # a key order needs the domain-contiguous order
        keys = np.arange(p.n, dtype=np.int64)
        kw = {"permute_domains": 0, "row_key": keys.ctypes.data}
    code, msg = _setup(n, rp, ci, va, pd, t, s, **kw)
    assert code == E.EINVAL, (case, code, msg)
    assert msg


def test_setup_without_gpu_reports_device_error(small):
    if gpu_available():
        pytest.skip("a GPU is present")
    p, dom = small
    code, msg = _setup(p.n, p.rowptr, p.colind, p.vals, dom, 4, 2)
    assert code == E.EDEVICE and msg


def test_null_arguments():
    assert E.lib.ecg_setup(None, 1, None, None, None, None, 1, 1, None) == E.EINVAL
    assert E.lib.ecg_solve(None, None, None, 1e-8, 10, None, None, None, None) == E.EINVAL
    assert E.lib.ecg_solve_ex(None, None, None, 1e-8, 10, None, 0, None) == E.EINVAL
    assert E.lib.ecg_sddmm(None, None, None, None) == E.EINVAL
    assert E.lib.ecg_spmm(None, None, None, 4) == E.EINVAL
    assert E.lib.ecg_spmm_noalloc(None, None, None, 4) == E.EINVAL
    assert E.lib.ecg_tsplit(None, None, None) == E.EINVAL
    assert E.lib.ecg_get_basis(None, None, None) == E.EINVAL
    assert E.lib.ecg_last_stats(None, None) == E.EINVAL
    E.lib.ecg_destroy(None)


@pytest.mark.parametrize("args", [(0, 4, 1, 1, 1, 1), (4, 4, 1, 5, 1, 1), (4, 4, 1, 0, 1, 1),
                                  (1 << 16, 1 << 16, 1, 1, 1, 1)])
def test_partition_rejects(args):
    buf = (ctypes.c_int32 * 4)()
    assert E.lib.ecg_partition_grid(*args, ctypes.addressof(buf), None) == E.EINVAL
    assert E.lib.ecg_partition_grid(4, 4, 1, 1, 1, 1, None, None) == E.EINVAL


def _morton_reference(nx, ny, nz):
    # bit b of x, y, z at bits 3b, 3b+1, 3b+2, written out bit by bit
    keys = np.zeros(nx * ny * nz, dtype=np.int64)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                key = 0
                for b in range(21):
                    key |= ((i >> b) & 1) << (3 * b)
                    key |= ((j >> b) & 1) << (3 * b + 1)
                    key |= ((k >> b) & 1) << (3 * b + 2)
                keys[i + nx * (j + ny * k)] = key
    return keys


@pytest.mark.parametrize("shape", [(8, 8, 8), (5, 3, 7), (37, 1, 1), (12, 9, 1)])
def test_grid_morton_keys(shape):
    # host code: against the bit-by-bit definition; distinct keys, and on a
    # power-of-two cube they are exactly 0 .. n-1 (a permutation)
    keys = E.grid_morton_keys(shape)
    assert np.array_equal(keys, _morton_reference(*shape))
    assert np.unique(keys).size == keys.size
    if shape == (8, 8, 8):
        assert np.array_equal(np.sort(keys), np.arange(512))


def test_grid_morton_keys_rejects():
    keys = np.zeros(8, dtype=np.int64)
    assert E.lib.ecg_grid_morton_keys(0, 2, 2, keys.ctypes.data) == E.EINVAL
    assert E.lib.ecg_grid_morton_keys(2, 2, 2, None) == E.EINVAL
    assert E.lib.ecg_grid_morton_keys(1 << 21, 1, 1, keys.ctypes.data) == E.EINVAL
