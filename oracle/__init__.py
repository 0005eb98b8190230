"""Python handle on the reference evaluator in oracle.cpp.

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product engine never imports it.

The evaluator computes the least fixpoint of a positive Datalog program
(Section 2) by semi-naive evaluation over sorted tuple vectors (Section 3),
with a naive evaluator beside it for cross-checks.  See oracle.cpp for the
exact algorithm.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.cpp into liboracle.so (g++, -O2, single thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp, cp, u32, u64 = ctypes.c_void_p, ctypes.c_char_p, ctypes.c_uint32, ctypes.c_uint64
        lib.orc_create.restype = vp
        lib.orc_destroy.argtypes = [vp]
        lib.orc_error.argtypes = [vp]
        lib.orc_error.restype = cp
        lib.orc_program.argtypes = [vp, cp]
        lib.orc_load.argtypes = [vp, cp, u32, vp, u64]
        lib.orc_run.argtypes = [vp, ctypes.c_int]
        lib.orc_size.argtypes = [vp, cp]
        lib.orc_size.restype = ctypes.c_int64
        lib.orc_export.argtypes = [vp, cp, vp, u64]
        lib.orc_rounds.argtypes = [vp]
        lib.orc_rounds.restype = u32
        lib.orc_delta_sizes.argtypes = [vp, vp, u32]
        lib.orc_seconds.argtypes = [vp]
        lib.orc_seconds.restype = ctypes.c_double
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


class Result:
    def __init__(self, relations, delta_sizes, seconds):
        self.relations = relations          # name -> (n, arity) uint32, rows sorted
        self.delta_sizes = delta_sizes      # per round, summed over relations
        self.seconds = seconds              # fixpoint wall time only

    @property
    def rounds(self) -> int:
        return len(self.delta_sizes)

    def __getitem__(self, name):
        return self.relations[name]


def evaluate(program: str, edb: dict, naive: bool = False, relations=None) -> Result:
    """Run `program` over `edb` (name -> list of column arrays) and return
    every relation's fixpoint as a row-sorted (n, arity) uint32 array."""
    lib = _load()
    h = lib.orc_create()
    try:
        def check(rc):
            if rc != 0:
                raise OracleError(lib.orc_error(h).decode())
        check(lib.orc_program(h, program.encode()))
        for name, cols in edb.items():
            rows = np.ascontiguousarray(np.stack([np.asarray(c, dtype=np.uint32) for c in cols], axis=1))
            check(lib.orc_load(h, name.encode(), rows.shape[1], rows.ctypes.data, rows.shape[0]))
        check(lib.orc_run(h, 1 if naive else 0))
        rounds = lib.orc_rounds(h)
        ds = np.zeros(max(rounds, 1), dtype=np.uint64)
        check(lib.orc_delta_sizes(h, ds.ctypes.data, rounds))
        names = relations if relations is not None else _relation_names(program, edb)
        out = {}
        for name in names:
            n = lib.orc_size(h, name.encode())
            if n < 0:
                raise OracleError(f"unknown relation {name}")
            arity = _arity_of(program, edb, name)
            buf = np.zeros((n, arity), dtype=np.uint32)
            check(lib.orc_export(h, name.encode(), buf.ctypes.data, n))
            out[name] = buf
        return Result(out, [int(x) for x in ds[:rounds]], lib.orc_seconds(h))
    finally:
        lib.orc_destroy(h)


def _atoms(program: str):
    import re
    text = "\n".join(line.split("%")[0] for line in program.splitlines())
    for m in re.finditer(r"([A-Za-z_][A-Za-z0-9_]*)\s*\(([^()]*)\)", text):
        yield m.group(1), len(m.group(2).split(","))


def _relation_names(program, edb):
    names = list(edb.keys())
    for n, _ in _atoms(program):
        if n not in names:
            names.append(n)
    return names


def _arity_of(program, edb, name):
    if name in edb:
        return len(edb[name])
    for n, a in _atoms(program):
        if n == name:
            return a
    raise OracleError(f"unknown relation {name}")
