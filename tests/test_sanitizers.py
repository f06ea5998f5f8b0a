"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host C code.

The oracle (oracle/ct_oracle.c) and the constraint compiler (csrc/compiler.cpp) are each built
with gcc's -fsanitize=address,undefined into a standalone driver (tests/helpers/san_*_main.*),
run over constraint sets with division and modulo by zero, negative values, chained comparisons,
min / max / abs / not, malformed text and deep nesting, and compared with the unsanitized code:
the oracle's enumeration, validity and every repair argmin with its ctypes build, the compiler's
return codes, bytecode and offsets with the library's ct_compile.  Any sanitizer report fails.
"""
import ctypes
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import core as ocore
from tests.test_oracle_repair import gap_space

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

EXTRA = {
    "zero_divisors": W.SpaceSpec("zero_divisors", {"a": [-3, -1, 0, 2, 5], "b": [0, 1, 2, 3], "c": [-2, 0, 7]},
                                 ["a // (b - 2) > -2 or c % b == 0", "not (a < b <= c) or abs(a) >= min(b, c)",
                                  "max(a, b, c) - min(a, c) != 4"]),
    "wide_values": W.SpaceSpec("wide_values", {"x": [-(1 << 40), -7, 0, 1 << 40], "y": [1, 3, 1 << 20]},
                               ["x * y > -2305843009213693952", "(x + y) % 7 != 3"]),
}


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, env=ENV, **kw)
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    return r


@pytest.fixture(scope="module")
def tools(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("san")
    oracle_exe = str(d / "san_oracle")
    r = subprocess.run(["gcc"] + SAN + [os.path.join(HERE, "helpers", "san_oracle_main.c"),
                                          os.path.join(ROOT, "oracle", "ct_oracle.c"), "-o", oracle_exe],
                       capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("gcc without sanitizer runtimes")
    assert r.returncode == 0, r.stderr
    # the compiler's own source, with an error reporter standing in for the library's
    src = d / "pkg" / "csrc"                   # the same layout: the source includes ../../include/ct.h
    src.mkdir(parents=True)
    (d / "include").mkdir()
    shutil.copy(os.path.join(ROOT, "include", "ct.h"), d / "include" / "ct.h")
    csrc = os.path.join(ROOT, "paper_2606_28372_amd", "csrc")
    for f in ("compiler.cpp", "ct_bytecode.h"):
        shutil.copy(os.path.join(csrc, f), src / f)
    (src / "ct_host.h").write_text("#pragma once\n#include <string>\n#include \"ct.h\"\n"
                                   "int ct_fail(int code, const std::string& msg);\n")
    compiler_exe = str(d / "san_compiler")
    r = subprocess.run(["g++", "-std=c++17"] + SAN + ["-I", os.path.join(ROOT, "include"), "-I", str(src),
                                                       str(src / "compiler.cpp"),
                                                       os.path.join(HERE, "helpers", "san_compiler_main.cpp"),
                                                       "-o", compiler_exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return d, oracle_exe, compiler_exe


@pytest.mark.parametrize("name", ["tiny", "gemm10", "gap", "bat_convolution", "zero_divisors", "wide_values"])
def test_oracle_under_sanitizers(tools, name):
    d, exe, _ = tools
    if name == "gap":
        osp = gap_space()
    elif name in EXTRA:
        osp = ocore.Space.from_spec(EXTRA[name]).enumerate()
    else:
        osp = ocore.Space.from_spec(W.space(name)).enumerate()
    rng = np.random.default_rng(3)
    n = 150
    cands = np.stack([rng.integers(0, r, n) for r in osp.radices], 1).astype(np.int64)
    pos = (cands << 16) + rng.integers(0, 65536, size=cands.shape)
    who = rng.integers(0, 2 ** 32, n)
    key, gen = 0x0123_4567_89AB_CDEF, 5
    n_cons = len(osp.constraints)
    vals = [osp.D] + osp.radices.tolist() + [len(osp._vals)] + osp._vals.tolist()
    vals += [n_cons, len(osp._expr)] + osp._expr.tolist() + osp._expr_off.tolist()[:n_cons]
    vals += [n] + cands.ravel().tolist() + pos.ravel().tolist() + who.tolist() + [key - (1 << 64) if key >= 1 << 63 else key, gen]
    inp, outp = d / f"{name}.in", d / f"{name}.out"
    inp.write_bytes(struct.pack(f"<{len(vals)}q", *vals))
    r = _run([exe, str(inp), str(outp)])
    assert r.returncode == 0, r.stderr[-3000:]
    blob = np.frombuffer(outp.read_bytes(), dtype=np.int64)
    n_words = (osp.n_cartesian + 63) // 64
    assert np.array_equal(blob[:n_words].view(np.uint64), osp.words)
    assert np.array_equal(blob[n_words:n_words + n].astype(bool), osp.valid_rows(cands))
    o = n_words + n
    for metric in range(5):
        want = osp.argmin(cands, metric, who=who.astype(np.uint32), key=key, gen=gen, pos_q16=pos)
        assert np.array_equal(blob[o:o + n], want), f"{name} metric {metric}"
        o += n


COMPILER_CASES = {name: (list(W.space(name).params.items()), W.space(name).constraints)
                  for name in ["tiny", "gemm13", "sparse16", "wide20"] + list(W.BAT_SPACES)}
COMPILER_CASES.update({k: (list(v.params.items()), v.constraints) for k, v in EXTRA.items()})
BAD = ["a +", "a == == 1", "nosuchname > 1", "(" * 40 + "a" + ")" * 40, "a" + " + a" * 40,
       "a * 99999999999999999999", "", "a // ", "min()", "a < < b", "abs(a, b)", "a @ b", "((a)",
       "a * a * a * a * a * a * a * a > 1"]


def compile_with_library(params, constraints):
    from paper_2606_28372_amd import _lib
    L = _lib.load()
    names = [p for p, _ in params]
    flat = np.ascontiguousarray([int(x) for _, v in params for x in v], dtype=np.int64)
    rad = np.ascontiguousarray([len(v) for _, v in params], dtype=np.uint32)
    cnames = (ctypes.c_char_p * len(names))(*[s.encode() for s in names])
    ccons = (ctypes.c_char_p * max(1, len(constraints)))(*[c.encode() for c in constraints])
    cap = 64 + 64 * sum(len(c) for c in constraints)
    code = np.zeros(cap, dtype=np.uint32)
    offs = np.zeros(len(constraints) + 1, dtype=np.uint32)
    used = ctypes.c_uint32(0)
    rc = L.ct_compile(cnames, len(names), flat.ctypes.data, rad.ctypes.data, ccons, len(constraints),
                      code.ctypes.data, cap, offs.ctypes.data, ctypes.byref(used))
    return rc, (code[: used.value].tolist() if rc == 0 else []), (offs.tolist() if rc == 0 else [])


def run_compiler(tools, tag, params, constraints):
    d, _, exe = tools
    lines = [str(len(params))] + [f"{n} {len(v)} " + " ".join(str(int(x)) for x in v) for n, v in params]
    lines += [str(len(constraints))] + list(constraints)
    inp, outp = d / f"c_{tag}.in", d / f"c_{tag}.out"
    inp.write_text("\n".join(lines) + "\n")
    r = _run([exe, str(inp), str(outp)])
    assert r.returncode == 0, r.stderr[-3000:]
    got = outp.read_text().split("\n")
    rc, used = int(got[0]), int(got[1])
    code = [int(x) for x in got[2].split()]
    offs = [int(x) for x in got[3].split()]
    assert len(code) == used
    return rc, code, offs


@pytest.mark.parametrize("name", sorted(COMPILER_CASES))
def test_compiler_under_sanitizers(tools, name):
    params, cons = COMPILER_CASES[name]
    assert run_compiler(tools, name, params, cons) == compile_with_library(params, cons)


def test_compiler_errors_under_sanitizers(tools):
    params = [("a", [1, 2, 3]), ("b", [-4, 0, 9])]
    for k, text in enumerate(BAD):
        got = run_compiler(tools, f"bad{k}", params, [text])
        assert got == compile_with_library(params, [text]), text
