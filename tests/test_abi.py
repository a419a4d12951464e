"""Host-only checks of the C ABI: the shared library loads, exports every
function declared in include/lbmibm.h, and its host-side argument checks
(buffer sizing) behave as documented.  No GPU call is made."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmibm.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1904_02108_amd import lbmibm
    return lbmibm


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ("lbm_buffer_sizes", "lbm_create", "lbm_destroy", "lbm_last_error",
                 "ibm_set_points", "ibm_force_iterate", "lbm_step", "lbm_read_fields",
                 "lbm_write_fields"):
        assert want in names


def test_library_exports_every_declared_symbol(L):
    lib = ct.CDLL(L.LIB_PATH)
    names = _declared_functions()
    assert names
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.ABI_FUNCTIONS) <= set(names)


def test_struct_layouts(L):
    # sizes fixed by the header's field list (x86-64 SysV alignment)
    assert ct.sizeof(L.lbm_params) == 4 * 8 + 8 * 2 + 8 * 18 + 8 * 3 + 8 + 8 * 3 + 8 + 4 + 4 + 8
    assert ct.sizeof(L.ibm_body) == 64
    assert ct.sizeof(L.ibm_stats) == 8 + 16 + 8 * 64
    assert ct.sizeof(L.lbm_fields) == 8 + 10 * 8


def test_buffer_sizes_scale(L):
    p = L.make_params((64, 32, 16), 0.6, max_points=1000, max_iter=5)
    s32 = L.lbm_buffer_sizes(p)
    ncell = 64 * 32 * 16
    assert s32[0] == 2 * 19 * ncell * 4
    assert s32[1] >= 2 * 3 * ncell * 4
    p16 = L.make_params((64, 32, 16), 0.6, storage=L.LBM_STORE_F16, max_points=1000, max_iter=5)
    assert L.lbm_buffer_sizes(p16)[0] == 2 * 19 * ncell * 2
    assert all(v % 256 == 0 for v in s32)


@pytest.mark.parametrize("bad", [dict(shape=(0, 4, 4), tau=0.6), dict(shape=(4, 4, 4), tau=0.5),
                                 dict(shape=(4, 4, 4), tau=0.6, bc=(0, 2, 0)),
                                 dict(shape=(4, 4, 4), tau=0.6, storage=7),
                                 dict(shape=(4, 4, 4), tau=0.6, forcing=3),
                                 dict(shape=(4, 4, 4), tau=0.6, max_iter=0),
                                 dict(shape=(4, 4, 4), tau=0.6, max_iter=65),
                                 dict(shape=(4, 4, 4), tau=0.6, max_points=-1),
                                 dict(shape=(2048, 2048, 1024), tau=0.6)])
def test_buffer_sizes_rejects(L, bad):
    kw = dict(bad)
    shape, tau = kw.pop("shape"), kw.pop("tau")
    with pytest.raises(L.LbmError) as ei:
        L.lbm_buffer_sizes(L.make_params(shape, tau, **kw))
    assert ei.value.status == L.LBM_ERR_ARG
    assert L.lbm_last_error(None)
