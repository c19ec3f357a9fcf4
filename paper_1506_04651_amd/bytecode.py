"""Compile right-hand sides written as arithmetic expressions into the
register programs of the bytecode model (RD_BYTECODE; format in include/rd.h).

    params = compile_model(["(-q*a - a*b + f*c)/mu", "(q*a - a*b + b*(1 - b))/eps", "b - c"],
                           species=["a", "b", "c"],
                           constants={"q": 2e-3, "f": 1.6, "mu": 1e-5, "eps": 1e-2})
    rd.reaction_step(u, dt, rtol, atol, rd.BYTECODE, params)

Expressions use + - * / ** (power), unary minus, exp() and log(), species
names, named constants and numeric literals.  Evaluation follows Python's
operator precedence and left-to-right association, one operation per
instruction, so the program rounds exactly like the expression evaluated in
FP64 without contraction.  Identical sub-expressions are computed once;
temporaries are packed into the 64 registers by their live ranges.
"""
from __future__ import annotations

import ast

import numpy as np

ADD, SUB, MUL, DIV, NEG, EXP, LOG, POW, OUT = range(1, 10)
REGS = 64
MAX_M = 16

_BIN = {ast.Add: ADD, ast.Sub: SUB, ast.Mult: MUL, ast.Div: DIV, ast.Pow: POW}
_FUN = {"exp": EXP, "log": LOG}


class CompileError(ValueError):
    pass


def compile_model(exprs, species, constants=None) -> np.ndarray:
    """Return the float64 params array of the register program computing
    f_i = exprs[i] for the given species (len(species) = m, 1 <= m <= 16)."""
    species = list(species)
    m = len(species)
    if not 1 <= m <= MAX_M or len(exprs) != m:
        raise CompileError(f"need 1..{MAX_M} species and one expression per species")
    constants = dict(constants or {})
    names = set(species) | set(constants)
    if len(names) != m + len(constants):
        raise CompileError("species and constant names must be distinct")

    const_vals: list[float] = []
    const_reg: dict[float | str, int] = {}

    def const(key, value):
        if key not in const_reg:
            const_vals.append(float(value))
            const_reg[key] = -len(const_vals)       # fixed up after counting
        return const_reg[key]

    # pass 1: SSA list of (op, a, b) over value ids; ids < 0 are constants,
    # ids 0..m-1 species, ids >= m temporaries in creation order
    ssa: list[tuple[int, int, int]] = []
    memo: dict[tuple, int] = {}

    def emit(op, a, b=0):
        key = (op, a, b)
        if key in memo:
            return memo[key]
        ssa.append(key)
        vid = m + len(ssa) - 1
        memo[key] = vid
        return vid

    def walk(node):
        if isinstance(node, ast.Expression):
            return walk(node.body)
        if isinstance(node, ast.BinOp) and type(node.op) in _BIN:
            a = walk(node.left)
            b = walk(node.right)
            return emit(_BIN[type(node.op)], a, b)
        if isinstance(node, ast.UnaryOp) and isinstance(node.op, ast.USub):
            return emit(NEG, walk(node.operand))
        if isinstance(node, ast.UnaryOp) and isinstance(node.op, ast.UAdd):
            return walk(node.operand)
        if isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and \
                node.func.id in _FUN and len(node.args) == 1 and not node.keywords:
            return emit(_FUN[node.func.id], walk(node.args[0]))
        if isinstance(node, ast.Name):
            if node.id in species:
                return species.index(node.id)
            if node.id in constants:
                return const(node.id, constants[node.id])
            raise CompileError(f"unknown name {node.id!r}")
        if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)) and \
                not isinstance(node.value, bool):
            return const(("lit", float(node.value)), node.value)
        raise CompileError(f"unsupported syntax: {ast.dump(node)}")

    outs = []
    for e in exprs:
        try:
            tree = ast.parse(e, mode="eval")
        except SyntaxError as err:
            raise CompileError(str(err)) from None
        outs.append(walk(tree))

    C = len(const_vals)
    base = m + C
    if base > REGS:
        raise CompileError("too many constants")

    # constants: id -k -> register m + k - 1
    def reg_of_input(vid):
        return m + (-vid) - 1 if vid < 0 else vid

    # an output that is a bare species or constant needs no temporary: OUT
    # reads it directly.  Live ranges of temporaries (SSA index -> last use).
    last_use = {}
    for i, (op, a, b) in enumerate(ssa):
        for v in ((a, b) if op in (ADD, SUB, MUL, DIV, POW) else (a,)):
            if v >= m:
                last_use[v] = i
    end = len(ssa)
    for v in outs:
        if v >= m:
            last_use[v] = end

    free = list(range(REGS - 1, base - 1, -1))   # pop() gives the lowest register
    where: dict[int, int] = {}
    code = []
    for i, (op, a, b) in enumerate(ssa):
        vid = m + i
        ra = where[a] if a >= m else reg_of_input(a)
        rb = (where[b] if b >= m else reg_of_input(b)) if op in (ADD, SUB, MUL, DIV, POW) else 0
        # operands whose last use is this instruction free their registers
        for v in ((a, b) if op in (ADD, SUB, MUL, DIV, POW) else (a,)):
            if v >= m and last_use.get(v) == i and v in where:
                free.append(where.pop(v))
                free.sort(reverse=True)
        if vid not in last_use:
            continue            # never used (cannot happen for reachable nodes)
        if not free:
            raise CompileError(f"program needs more than {REGS} registers")
        rd = free.pop()
        where[vid] = rd
        code.append((op, rd, ra, rb))
    for i, v in enumerate(outs):
        code.append((OUT, i, where[v] if v >= m else reg_of_input(v), 0))

    prog = [float(len(code)), float(C)] + const_vals
    for ins in code:
        prog += [float(x) for x in ins]
    return np.array(prog, dtype=np.float64)
