"""Pins the oracle's constraint evaluation against Python's own eval.

A configuration is a solution iff every constraint holds (Section IV-A).
Constraints are Python integer expressions; the oracle walks its own
expression trees in C.  Here random expressions are evaluated by Python and
by the oracle: for a Python value v the oracle must accept `(e) == v` and
reject `(e) == v + 1`; where Python raises (division by zero) the oracle must
reject the constraint whatever it is compared with.
"""
import hypothesis.strategies as st
import numpy as np
import pytest
from hypothesis import given, settings, HealthCheck

from oracle import core

NAMES = ["a", "b", "c"]


def exprs(depth):
    leaf = st.one_of(st.integers(-9, 9).map(str), st.sampled_from(NAMES))
    if depth == 0:
        return leaf
    sub = exprs(depth - 1)
    binop = st.tuples(sub, st.sampled_from(["+", "-", "*", "//", "%"]), sub).map(lambda t: f"({t[0]} {t[1]} {t[2]})")
    cmp_ = st.tuples(sub, st.sampled_from(["<", "<=", ">", ">=", "==", "!="]), sub,
                     st.sampled_from(["<", "<=", "==", "!="]), sub).map(
        lambda t: f"({t[0]} {t[1]} {t[2]} {t[3]} {t[4]})")
    cmp2 = st.tuples(sub, st.sampled_from(["<", ">=", "=="]), sub).map(lambda t: f"({t[0]} {t[1]} {t[2]})")
    boolop = st.tuples(sub, st.sampled_from(["and", "or"]), sub).map(lambda t: f"({t[0]} {t[1]} {t[2]})")
    unary = st.tuples(st.sampled_from(["-", "not ", "abs"]), sub).map(
        lambda t: f"abs({t[1]})" if t[0] == "abs" else f"({t[0]}{t[1]})")
    call = st.tuples(st.sampled_from(["min", "max"]), sub, sub, sub).map(lambda t: f"{t[0]}({t[1]}, {t[2]}, {t[3]})")
    return st.one_of(leaf, binop, cmp_, cmp2, boolop, unary, call)


def py_value(e, env):
    try:
        return int(eval(e, {"__builtins__": {}, "abs": abs, "min": min, "max": max}, dict(env))), False
    except ZeroDivisionError:
        return None, True


def oracle_holds(constraint, env):
    sp = core.Space(NAMES, [[env[n]] for n in NAMES], [constraint])
    return bool(sp.valid_rows(np.zeros((1, 3), dtype=np.int32))[0])


@settings(max_examples=400, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(e=exprs(3), a=st.integers(-6, 6), b=st.integers(-6, 6), c=st.integers(-6, 6))
def test_random_expressions_match_python(e, a, b, c):
    env = {"a": a, "b": b, "c": c}
    v, raised = py_value(e, env)
    if raised:
        assert not oracle_holds(f"({e}) == 0", env)
        assert not oracle_holds(f"({e}) != 0", env)
    else:
        assert oracle_holds(f"({e}) == {v}", env)
        assert not oracle_holds(f"({e}) == {v + 1}", env)
        assert oracle_holds(e, env) == bool(v)


@pytest.mark.parametrize("e,env,expect", [
    ("7 // -2 == -4", {}, True),                 # floor, not truncation
    ("-7 % 3 == 2", {}, True),                   # sign of the divisor
    ("7 % -3 == -2", {}, True),
    ("a == 0 or 5 // a > 1", {"a": 0}, True),    # 'or' short-circuits past the division
    ("a != 0 and 5 // a > 1", {"a": 0}, False),  # 'and' short-circuits
    ("5 // a > 1 or a == 0", {"a": 0}, False),   # division evaluated first raises -> constraint false
    ("(2 and 3) == 3", {}, True),                # 'and' returns its last operand
    ("(0 or 4) == 4", {}, True),
    ("1 < a < 3", {"a": 2}, True),
    ("1 < a < 3", {"a": 3}, False),
    ("3 > a < 5 // a", {"a": 0}, False),         # second comparison's operand raises
    ("3 < a < 5 // a", {"a": 0}, False),         # first comparison false: no evaluation of 5 // a
    ("not a", {"a": 0}, True),
    ("-a * 2 == -6", {"a": 3}, True),            # unary minus binds tighter than *
    ("not a == 3", {"a": 3}, False),             # 'not' binds looser than ==
])
def test_python_semantics_cases(e, env, expect):
    names = NAMES
    full = {n: env.get(n, 1) for n in names}
    assert oracle_holds(e, full) == expect
    v, raised = py_value(e, full)
    assert (bool(v) if not raised else False) == expect   # the case table itself follows Python


def test_overflow_is_reported_not_wrapped():
    sp = core.Space(["a"], [[2 ** 40]], ["a * a * a > 0"])
    with pytest.raises(OverflowError):
        sp.valid_rows(np.zeros((1, 1), dtype=np.int32))
