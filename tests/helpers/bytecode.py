"""Test-side reader of libct's constraint bytecode (documented in ct_bytecode.h).

Evaluates one program per constraint with the documented stack semantics so
that the CPU tests can check the compiler's output against Python eval
without a GPU.  It mirrors the documented format, not the device code.
"""
OPS = dict(PARAM=1, CONST=2, CONST64=3, NEG=4, ABS=5, NOT=6, ADD=7, SUB=8, MUL=9, FDIV=10, MOD=11, MIN=12, MAX=13,
           LT=14, LE=15, GT=16, GE=17, EQ=18, NE=19, AND=20, OR=21)
N = {v: k for k, v in OPS.items()}


def run(code, start, end, pv):
    """Returns (value, raised)."""
    st = []   # (value, raised)
    pc = start
    while pc < end:
        w = int(code[pc]); pc += 1
        op, imm = w & 0xFF, (w >> 8) - (1 << 24 if w >> 31 else 0)
        name = N[op]
        if name == "PARAM":
            st.append((pv[imm], False))
        elif name == "CONST":
            st.append((imm, False))
        elif name == "CONST64":
            v = int(code[pc]) | (int(code[pc + 1]) << 32); pc += 2
            st.append((v - (1 << 64) if v >> 63 else v, False))
        elif name in ("NEG", "ABS", "NOT"):
            a, e = st.pop()
            st.append(({"NEG": -a, "ABS": abs(a), "NOT": int(a == 0)}[name], e))
        else:
            (b, eb), (a, ea) = st.pop(), st.pop()
            if name == "AND":
                st.append((0, True) if ea else ((a, False) if a == 0 else (b, eb)))
                continue
            if name == "OR":
                st.append((0, True) if ea else ((a, False) if a != 0 else (b, eb)))
                continue
            e = ea or eb
            if name in ("FDIV", "MOD") and b == 0:
                st.append((0, True))
                continue
            r = {"ADD": lambda: a + b, "SUB": lambda: a - b, "MUL": lambda: a * b, "FDIV": lambda: a // b,
                 "MOD": lambda: a % b, "MIN": lambda: min(a, b), "MAX": lambda: max(a, b),
                 "LT": lambda: int(a < b), "LE": lambda: int(a <= b), "GT": lambda: int(a > b),
                 "GE": lambda: int(a >= b), "EQ": lambda: int(a == b), "NE": lambda: int(a != b)}[name]()
            st.append((r, e))
    assert len(st) == 1
    return st[0][0], st[0][1]
