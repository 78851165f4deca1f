"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, and rejects invalid arguments before any device
work (no compute call is made here)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dps.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dps_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2405_16788_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2405_16788_amd.build import build
        build()
    return binding.load()


def test_header_declares_expected_calls():
    names = _declared()
    for n in ("dps_build", "dps_set_attributes", "dps_query", "dps_query_counts", "dps_adjoint",
              "dps_adjoint_zero", "dps_adjoint_accumulate", "dps_adjoint_finalize", "dps_export_tree",
              "dps_tree_info", "dps_check", "dps_destroy", "dps_status_string", "dps_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2405_16788_amd import binding
    names = _declared()
    for n in names:
        assert hasattr(lib, n), f"{n} missing from libdps.so"
    assert set(names) == set(binding.EXPORTED)


def test_status_strings(lib):
    assert lib.dps_status_string(0) == b"ok"
    assert lib.dps_status_string(1) == b"invalid argument"
    assert lib.dps_status_string(4) == b"invalid tree handle"
    assert lib.dps_status_string(99) == b"unknown status"


def _build(lib, p=1, n=1, A=1, attrs=1, M=10, C=4, leaf=16, storage=0, out=True):
    h = ct.c_void_p(123)
    fake = lambda b: ct.c_void_p(0x1000) if b else None  # never dereferenced: rejected first
    rc = lib.dps_build(fake(p), fake(n), fake(A), fake(attrs), M, C, leaf, storage, None,
                       ct.byref(h) if out else None)
    return rc, h


@pytest.mark.parametrize("kw", [
    dict(M=0), dict(M=-5), dict(M=1 << 31), dict(C=0), dict(C=33), dict(leaf=0), dict(leaf=257),
    dict(storage=7), dict(p=0), dict(n=0), dict(A=0), dict(attrs=0),
])
def test_build_rejects_invalid_arguments(lib, kw):
    rc, h = _build(lib, **kw)
    assert rc == 1, lib.dps_last_error()
    assert h.value is None  # *out cleared
    assert lib.dps_last_error().startswith(b"dps_build")


def test_build_rejects_null_out(lib):
    rc, _ = _build(lib, out=False)
    assert rc == 1


def test_calls_on_unknown_handles(lib):
    bogus = ct.c_void_p(0xdead0000)
    x = ct.c_void_p(0x1000)
    assert lib.dps_query(None, x, 4, 2.0, 0.1, x, None, None) == 4
    assert lib.dps_query(bogus, x, 4, 2.0, 0.1, x, None, None) == 4
    assert lib.dps_set_attributes(bogus, x, None) == 4
    assert lib.dps_adjoint_zero(bogus, None) == 4
    assert lib.dps_adjoint_accumulate(bogus, x, 4, 2.0, 0.1, x, None, None) == 4
    assert lib.dps_adjoint_finalize(bogus, x, None) == 4
    assert lib.dps_adjoint(bogus, x, 4, 2.0, 0.1, x, x, None, None) == 4
    assert lib.dps_export_tree(bogus, None, None, None, None, None, None) == 4
    assert lib.dps_check(bogus, None) == 4
    n = ct.c_int64()
    assert lib.dps_tree_info(bogus, ct.byref(n), None, None, None, None) == 4
    lib.dps_destroy(None)   # no-op
    lib.dps_destroy(bogus)  # unknown handles are ignored


def test_limits_validate_without_a_device(lib):
    bogus = ct.c_void_p(0xdead0000)
    assert lib.dps_set_step_limit(bogus, 5) == 4
    assert lib.dps_set_step_limit(None, 0) == 4
    assert lib.dps_set_memory_limit(-1) == 1
    assert lib.dps_last_error().startswith(b"dps_set_memory_limit")
    assert lib.dps_set_memory_limit(1 << 30) == 0
    assert lib.dps_set_memory_limit(0) == 0
