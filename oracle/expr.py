"""Oracle-side reading of constraint strings -- TEST INFRASTRUCTURE ONLY.

Constraints are Python integer expressions over the parameter names (the
Kernel Tuner convention used throughout Section II's example, e.g. the
bound on block_x*block_y).  This module turns each one into the oracle's own
prefix-encoded expression tree, which ct_oracle.c walks recursively with
Python semantics.  It is deliberately independent of the GPU library's
constraint compiler: it uses Python's own parser and keeps the tree shape
one-to-one with the source (no constant folding, no rewriting).
"""
from __future__ import annotations

import ast
from typing import Dict, List

T_NUM, T_PARAM, T_NEG, T_NOT, T_ABS = 1, 2, 3, 5, 6
T_ADD, T_SUB, T_MUL, T_FDIV, T_MOD = 10, 11, 12, 13, 14
T_MIN, T_MAX, T_CMP, T_AND, T_OR = 20, 21, 30, 40, 41
CMP = {ast.Lt: 0, ast.LtE: 1, ast.Gt: 2, ast.GtE: 3, ast.Eq: 4, ast.NotEq: 5}
BIN = {ast.Add: T_ADD, ast.Sub: T_SUB, ast.Mult: T_MUL,
       ast.FloorDiv: T_FDIV, ast.Mod: T_MOD}


class Unsupported(ValueError):
    pass


def _enc(node: ast.AST, index: Dict[str, int], out: List[int]) -> None:
    if isinstance(node, ast.Constant) and isinstance(node.value, (bool, int)):
        out += [T_NUM, int(node.value)]
    elif isinstance(node, ast.Name):
        if node.id in index:
            out += [T_PARAM, index[node.id]]
        elif node.id in ("True", "False"):
            out += [T_NUM, int(node.id == "True")]
        else:
            raise Unsupported(f"unknown name {node.id!r}")
    elif isinstance(node, ast.UnaryOp):
        if isinstance(node.op, ast.UAdd):
            _enc(node.operand, index, out)
        elif isinstance(node.op, ast.USub):
            out.append(T_NEG)
            _enc(node.operand, index, out)
        elif isinstance(node.op, ast.Not):
            out.append(T_NOT)
            _enc(node.operand, index, out)
        else:
            raise Unsupported(ast.dump(node.op))
    elif isinstance(node, ast.BinOp):
        if type(node.op) not in BIN:
            raise Unsupported(ast.dump(node.op))
        out.append(BIN[type(node.op)])
        _enc(node.left, index, out)
        _enc(node.right, index, out)
    elif isinstance(node, ast.BoolOp):
        out += [T_AND if isinstance(node.op, ast.And) else T_OR, len(node.values)]
        for v in node.values:
            _enc(v, index, out)
    elif isinstance(node, ast.Compare):
        out += [T_CMP, len(node.ops) + 1]
        for op in node.ops:
            if type(op) not in CMP:
                raise Unsupported(ast.dump(op))
            out.append(CMP[type(op)])
        _enc(node.left, index, out)
        for c in node.comparators:
            _enc(c, index, out)
    elif isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and not node.keywords:
        f = node.func.id
        if f == "abs" and len(node.args) == 1:
            out.append(T_ABS)
            _enc(node.args[0], index, out)
        elif f in ("min", "max") and len(node.args) >= 2:
            out += [T_MIN if f == "min" else T_MAX, len(node.args)]
            for a in node.args:
                _enc(a, index, out)
        else:
            raise Unsupported(f"call {f}")
    else:
        raise Unsupported(ast.dump(node))


def encode(constraint: str, names: List[str]) -> List[int]:
    """Prefix encoding of one constraint expression."""
    tree = ast.parse(constraint.strip(), mode="eval")
    out: List[int] = []
    _enc(tree.body, {n: i for i, n in enumerate(names)}, out)
    return out
