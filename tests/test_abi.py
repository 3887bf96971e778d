"""The C ABI without a GPU: the library loads, exports every function include/copa.h declares,
and rejects bad arguments on the host before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1803_04572_amd import copa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "copa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(copa_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(copa.LIB_PATH):
        pytest.skip("libcopa.so not built (run __graft_entry__.build())")
    return copa.lib()


def test_every_declared_symbol_is_exported(lib):
    declared = _header_functions()
    assert set(declared) == set(copa.SYMBOLS), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings_and_rank_table(lib):
    assert copa.status_name(copa.EINVAL) == "COPA_EINVAL"
    assert copa.status_name(copa.ENUMERIC) == "COPA_ENUMERIC"
    for R in (5, 10, 15, 20, 40):
        assert lib.copa_rank_supported(R) == 1
    assert lib.copa_rank_supported(0) == 0
    assert lib.copa_rank_supported(1000) == 0
    assert lib.copa_kernel_name(0).decode() == "pass1"
    assert lib.copa_kernel_name(99).decode() == "unknown"


def _create(lib, t, o):
    h = ctypes.c_void_p()
    st = lib.copa_plan_create(ctypes.byref(t) if t is not None else None,
                              ctypes.byref(o) if o is not None else None, None, 0, None,
                              ctypes.byref(h))
    return st, h


def test_host_side_rejections(lib):
    fake = ctypes.c_void_p(16)  # never dereferenced: every case below fails on the host first
    t = copa.CopaTensor(K=4, J=3, S=6, nnz=10, subj_ptr=fake, row_ptr=fake, col=fake, val=fake,
                        days=fake, l=7)
    o = copa.CopaOptions(R=10, inner_iters=5, prox_H=0, prox_W=1, prox_V=2, lambda_V=0.1)
    assert _create(lib, None, o)[0] == copa.EINVAL
    assert _create(lib, t, None)[0] == copa.EINVAL
    bad = copa.CopaOptions(R=0, inner_iters=5)
    assert _create(lib, t, bad)[0] == copa.EINVAL
    bad = copa.CopaOptions(R=10, inner_iters=0)
    assert _create(lib, t, bad)[0] == copa.EINVAL
    bad = copa.CopaOptions(R=10, inner_iters=5, prox_V=9)
    assert _create(lib, t, bad)[0] == copa.EINVAL
    bad = copa.CopaOptions(R=10, inner_iters=5, lambda_V=-1.0)
    assert _create(lib, t, bad)[0] == copa.EINVAL
    bad = copa.CopaOptions(R=11, inner_iters=5)
    st, _ = _create(lib, t, bad)
    assert st == copa.EUNSUPPORTED and "R=11" in copa.last_error()
    t9 = copa.CopaTensor(K=4, J=3, S=6, nnz=10, subj_ptr=fake, row_ptr=fake, col=fake, val=fake,
                         days=fake, l=9)
    assert _create(lib, t9, o)[0] == copa.EUNSUPPORTED
    tneg = copa.CopaTensor(K=-1, J=3, S=6, nnz=10, subj_ptr=fake, row_ptr=fake, col=fake,
                           val=fake, days=fake, l=0)
    assert _create(lib, tneg, o)[0] == copa.EINVAL
    tnull = copa.CopaTensor(K=4, J=3, S=6, nnz=10, subj_ptr=None, row_ptr=fake, col=fake,
                            val=fake, days=fake, l=0)
    assert _create(lib, tnull, o)[0] == copa.EINVAL
    tdays = copa.CopaTensor(K=4, J=3, S=6, nnz=10, subj_ptr=fake, row_ptr=fake, col=fake,
                            val=fake, days=None, l=7)
    assert _create(lib, tdays, o)[0] == copa.EINVAL
    # calls on a NULL plan
    assert lib.copa_fit(None, None, 1, None, None, None) == copa.EINVAL
    assert lib.copa_mttkrp_last(None, None, None, None, None) == copa.EINVAL
    assert lib.copa_plan_basis(None, None, None, None) == copa.EINVAL
    assert lib.copa_set_timing(None, 1) == copa.EINVAL
    lib.copa_plan_destroy(None)


def test_product_path_has_no_oracle_dependency():
    """The library's Python binding and sources never reach the oracle."""
    pkg = os.path.join(ROOT, "paper_1803_04572_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", text, flags=re.M), f
                assert "copa_oracle" not in text, f
