"""Read the plain-text fixtures under tests/golden (entries typed from the paper)."""
from __future__ import annotations

import ast
import operator
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

_OPS = {ast.Add: operator.add, ast.Sub: operator.sub, ast.Mult: operator.mul,
        ast.Div: operator.truediv, ast.Pow: operator.pow, ast.USub: operator.neg,
        ast.UAdd: operator.pos}


def _eval(node, env):
    if isinstance(node, ast.Expression):
        return _eval(node.body, env)
    if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
        return float(node.value)
    if isinstance(node, ast.Name):
        return env[node.id]
    if isinstance(node, ast.BinOp) and type(node.op) in _OPS:
        return _OPS[type(node.op)](_eval(node.left, env), _eval(node.right, env))
    if isinstance(node, ast.UnaryOp) and type(node.op) in _OPS:
        return _OPS[type(node.op)](_eval(node.operand, env))
    raise ValueError(f"unsupported fixture expression: {ast.dump(node)}")


def evaluate(expr: str, env: dict) -> float:
    """Arithmetic only: numbers, the names in env, + - * / and ^ (power)."""
    return _eval(ast.parse(expr.replace("^", "**"), mode="eval"), env)


def read_lines(name: str) -> list[str]:
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.strip() for ln in fh if ln.strip() and not ln.startswith("#")]


def read_matrix(name: str, env: dict) -> np.ndarray:
    rows = [ln.split() for ln in read_lines(name)]
    return np.array([[evaluate(tok, env) for tok in r] for r in rows])


def read_vector(name: str, env: dict) -> np.ndarray:
    return np.array([evaluate(ln, env) for ln in read_lines(name)])
