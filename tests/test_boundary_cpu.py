"""CPU checks of the C-ABI library: it loads, exports every function that
include/ct.h declares, and its constraint compiler (host-only, no GPU) emits
bytecode whose documented semantics match Python's on random expressions."""
import ctypes
import os
import re

import hypothesis.strategies as st
import numpy as np
import pytest
from hypothesis import given, settings, HealthCheck

from paper_2606_28372_amd import _lib, compile_constraints, CtError
from tests.helpers import bytecode
from tests.test_oracle_expr import exprs, py_value

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "ct.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|void|double|char\s*\*|const char\s*\*)\s*\*?\s*(ct_\w+)\s*\(",
                                 src, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = _lib.load()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"
    assert lib.ct_version() == 2


def eval_compiled(code, offs, k, pv):
    return bytecode.run(code, int(offs[k]), int(offs[k + 1]), pv)


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(e=exprs(3), a=st.integers(-6, 6), b=st.integers(-6, 6), c=st.integers(-6, 6))
def test_compiled_programs_follow_python(e, a, b, c):
    env = {"a": a, "b": b, "c": c}
    code, offs = compile_constraints(["a", "b", "c"], [[a], [b], [c]], [e])
    v, raised = py_value(e, env)
    got, graised = eval_compiled(code, offs, 0, [a, b, c])
    if raised:
        assert graised
    else:
        assert not graised and got == v


@pytest.mark.parametrize("bad,code", [
    ("a / 2 > 1", _lib.CT_ESYNTAX), ("a ** 2 > 1", _lib.CT_ESYNTAX), ("zz > 1", _lib.CT_ESYNTAX),
    ("a > 1.5", _lib.CT_ESYNTAX), ("'x' == a", _lib.CT_ESYNTAX), ("foo(a) > 1", _lib.CT_ESYNTAX),
    ("a << 2 > 1", _lib.CT_ESYNTAX), ("(a > 1", _lib.CT_ESYNTAX), ("a > 1)", _lib.CT_ESYNTAX),
    ("a * a * a * a * a > 1", _lib.CT_EOVERFLOW),
])
def test_compile_errors(bad, code):
    with pytest.raises(CtError) as ei:
        compile_constraints(["a"], [[1, 2 ** 20]], [bad])
    assert ei.value.code == code


def test_large_constants_and_precedence():
    code, offs = compile_constraints(["a"], [[3]], ["a * 10_000_000_000 == 30000000000", "-a * 2 == -6",
                                                    "not a == 4", "0x10 + a == 19", "True + a == 4"])
    for k in range(5):
        assert eval_compiled(code, offs, k, [3]) == (1, False)


def test_server_needs_device_and_objective():
    """Server creation fails cleanly without an objective callback, and without a HIP device."""
    import torch
    from paper_2606_28372_amd import CtError, Server, _lib
    cfg = _lib.ct_server_config(hbm_budget=1 << 20, max_active=4)
    h = ctypes.c_void_p()
    assert _lib.load().ct_server_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.CT_EINVAL
    cfg.max_active = 0
    assert _lib.load().ct_server_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.CT_EINVAL
    if not torch.cuda.is_available():
        with pytest.raises(CtError) as e:
            Server(lambda rid, nv: None, hbm_budget=1 << 20)
        assert e.value.code == _lib.CT_EDEVICE


def test_batch_tuning_null_handles():
    """The tuning entry points reject a null batch before touching the device."""
    from paper_2606_28372_amd import _lib
    lib = _lib.load()
    assert lib.ct_batch_set_tuning(None, 4096, 16, 8192, 0) == _lib.CT_EINVAL
    assert lib.ct_batch_tuning(None, None, None, None, None, None) == _lib.CT_EINVAL
    assert lib.ct_batch_autotune(None, 1, 1, 0, None) == _lib.CT_EINVAL


# ---------------------------------------------------------------------------
# ct_space_build rejects malformed constraint programs on the host, before it
# touches a device (CT_EINVAL); a well-formed program then needs the device.
# ---------------------------------------------------------------------------
def _w(op, imm=0):
    return ((imm & 0xFFFFFF) << 8) | op


OP = bytecode.OPS


def _build(progs, radices=(4, 3, 5), offsets=None):
    lib = _lib.load()
    values = np.ascontiguousarray([v for r in radices for v in range(1, r + 1)], dtype=np.int64)
    rad = np.ascontiguousarray(radices, dtype=np.uint32)
    flat, offs = [], [0]
    for p in progs:
        flat += p
        offs.append(len(flat))
    code = np.ascontiguousarray(flat or [0], dtype=np.uint32)
    offs = np.ascontiguousarray(offs if offsets is None else offsets, dtype=np.uint32)
    h = ctypes.c_void_p()
    rc = lib.ct_space_build(values.ctypes.data, rad.ctypes.data, len(radices), code.ctypes.data, offs.ctypes.data,
                            len(progs), None, ctypes.byref(h))
    if rc == 0:
        lib.ct_space_free(h)
    return rc, lib.ct_last_error().decode()


@pytest.mark.parametrize("name,prog,why", [
    ("binary underflow", [_w(OP["CONST"], 1), _w(OP["ADD"])], "underflow"),
    ("unary underflow", [_w(OP["NEG"])], "underflow"),
    ("depth 17", [_w(OP["CONST"], 1)] * 17 + [_w(OP["ADD"])] * 16, "deeper than 16"),
    ("opcode 0", [_w(OP["CONST"], 1), _w(OP["CONST"], 1), _w(0)], "unknown opcode"),
    ("opcode 22", [_w(OP["CONST"], 1), _w(OP["CONST"], 1), _w(22)], "unknown opcode"),
    ("opcode 255", [_w(OP["CONST"], 1), _w(255)], "unknown opcode"),
    ("parameter id = n", [_w(OP["PARAM"], 3)], "parameter id"),
    ("negative parameter id", [_w(OP["PARAM"], -1)], "parameter id"),
    ("truncated CONST64", [_w(OP["CONST64"]), 7], "truncated"),
    ("two values left", [_w(OP["CONST"], 1), _w(OP["CONST"], 2)], "exactly one value"),
    ("empty program", [], "exactly one value"),
])
def test_space_build_rejects_malformed_bytecode(name, prog, why):
    rc, msg = _build([[_w(OP["PARAM"], 0), _w(OP["CONST"], 2), _w(OP["GT"])], prog])
    assert rc == _lib.CT_EINVAL, name
    assert "program 1" in msg and why in msg, msg


@pytest.mark.parametrize("radices,why", [
    ((), "parameters"), (tuple([2] * 33), "parameters"), ((4, 0, 5), "radix"), ((4, 256, 5), "radix"),
    ((255,) * 6 + (6,), "2^46"),
])
def test_space_build_rejects_bad_sizes(radices, why):
    rc, msg = _build([], radices=radices)
    assert rc == _lib.CT_EINVAL and why in msg, msg


def test_space_build_rejects_descending_offsets():
    good = [_w(OP["CONST"], 1)]
    rc, msg = _build([good, good], offsets=[0, 1, 0])
    assert rc == _lib.CT_EINVAL and "ascending" in msg, msg


def test_space_build_accepts_depth_16_then_needs_a_device():
    """Sixteen values on the stack is the documented limit: the program passes validation, so
    without a GPU the build stops at the device check instead."""
    import torch
    prog = [_w(OP["CONST"], 1)] * 16 + [_w(OP["ADD"])] * 15
    rc, msg = _build([prog, [_w(OP["PARAM"], 2), _w(OP["CONST64"]), 5, 0, _w(OP["LT"])]])
    if torch.cuda.is_available():
        assert rc == 0, msg
    else:
        assert rc == _lib.CT_EDEVICE, msg
