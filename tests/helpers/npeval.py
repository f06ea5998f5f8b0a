"""Vectorised numpy evaluation of constraint strings (a third, independent engine).

Used only to brute-force valid-set sizes of medium spaces in the tests.
'and'/'or'/'not' are evaluated as boolean operations, which matches Python
for the constraint strings used here because every operand of a boolean
operator in them is itself a comparison or a boolean.
"""
import ast

import numpy as np


def _ev(node, env):
    if isinstance(node, ast.Constant):
        return np.int64(node.value)
    if isinstance(node, ast.Name):
        return env[node.id]
    if isinstance(node, ast.BoolOp):
        vals = [_ev(v, env) != 0 for v in node.values]
        out = vals[0]
        for v in vals[1:]:
            out = (out & v) if isinstance(node.op, ast.And) else (out | v)
        return out
    if isinstance(node, ast.UnaryOp):
        x = _ev(node.operand, env)
        if isinstance(node.op, ast.USub):
            return -x
        if isinstance(node.op, ast.Not):
            return x == 0
        return x
    if isinstance(node, ast.BinOp):
        a, b = _ev(node.left, env), _ev(node.right, env)
        op = type(node.op)
        if op is ast.Add:
            return a + b
        if op is ast.Sub:
            return a - b
        if op is ast.Mult:
            return a * b
        assert np.all(b != 0), "division by zero not handled by this helper"
        if op is ast.FloorDiv:
            return np.floor_divide(a, b)
        if op is ast.Mod:
            return np.mod(a, b)
    if isinstance(node, ast.Compare):
        out, left = None, _ev(node.left, env)
        for op, c in zip(node.ops, node.comparators):
            right = _ev(c, env)
            r = {ast.Lt: np.less, ast.LtE: np.less_equal, ast.Gt: np.greater, ast.GtE: np.greater_equal,
                 ast.Eq: np.equal, ast.NotEq: np.not_equal}[type(op)](left, right)
            out = r if out is None else (out & r)
            left = right
        return out
    if isinstance(node, ast.Call):
        args = [_ev(a, env) for a in node.args]
        f = {"min": np.minimum, "max": np.maximum}.get(node.func.id)
        if node.func.id == "abs":
            return np.abs(args[0])
        out = args[0]
        for a in args[1:]:
            out = f(out, a)
        return out
    raise NotImplementedError(ast.dump(node))


def valid_mask(names, values, constraints):
    """Boolean mask over the Cartesian space in linear-index order (last parameter fastest)."""
    grids = np.meshgrid(*[np.asarray(v, dtype=np.int64) for v in values], indexing="ij")
    env = {n: g.ravel() for n, g in zip(names, grids)}
    ok = np.ones(grids[0].size, dtype=bool)
    for c in constraints:
        ok &= np.asarray(_ev(ast.parse(c, mode="eval").body, env) != 0)
    return ok
