"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/fv.h declares, and rejects bad relations and rules
before any device work."""
import ctypes
import os
import re

import pytest

from paper_2501_13051_amd import fv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fv_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert set(declared_functions()) == set(fv.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = fv.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def _ctx():
    L = fv.lib()
    h = ctypes.c_void_p()
    assert L.fv_ctx_create(ctypes.byref(h), None) == 0
    return L, h


def test_relation_and_rule_validation_without_device():
    L, h = _ctx()
    try:
        r = ctypes.c_uint32()
        assert L.fv_relation_create(h, b"edge", 2, ctypes.byref(r)) == 0
        e = r.value
        assert L.fv_relation_create(h, b"path", 2, ctypes.byref(r)) == 0
        p = r.value
        assert L.fv_relation_create(h, b"edge", 2, ctypes.byref(r)) == -1       # duplicate name
        assert L.fv_relation_create(h, b"bad", 4, ctypes.byref(r)) == -3        # arity 4
        f = ctypes.c_uint32()
        assert L.fv_relation_find(h, b"path", ctypes.byref(f)) == 0 and f.value == p

        def rule(head_terms, body):
            keep = []

            def atom(rel, ts):
                arr = (fv.Term * len(ts))(*[fv.Term(v, c) for v, c in ts])
                keep.append(arr)
                return fv.Atom(rel, len(ts), arr)
            R = fv.Rule()
            R.head = atom(p, head_terms)
            R.body = (fv.Atom * len(body))(*[atom(rel, ts) for rel, ts in body])
            R.n_body = len(body)
            R.n_neq = 0
            return R, keep

        ok, k1 = rule([(0, 0), (1, 0)], [(e, [(0, 0), (1, 0)])])
        assert L.fv_add_rule(h, ctypes.byref(ok)) == 0
        unsafe, k2 = rule([(0, 0), (2, 0)], [(e, [(0, 0), (1, 0)])])
        assert L.fv_add_rule(h, ctypes.byref(unsafe)) == -4                   # FV_EUNSAFE
        assert b"head variable" in L.fv_last_error(h)
        arity, k3 = rule([(0, 0), (1, 0)], [(e, [(0, 0)])])
        arity.body[0].arity = 1
        assert L.fv_add_rule(h, ctypes.byref(arity)) == -3                    # FV_EARITY
        reserved, k4 = rule([(0, 0), (0xFFFFFFFF, 1)], [(e, [(0, 0), (1, 0)])])
        assert L.fv_add_rule(h, ctypes.byref(reserved)) == -7                 # FV_ERESERVED
        bigvar, k5 = rule([(0, 0), (16, 0)], [(e, [(0, 0), (16, 0)])])
        assert L.fv_add_rule(h, ctypes.byref(bigvar)) == -1                   # variable index > 15
        n = ctypes.c_uint64()
        assert L.fv_export(h, p, None, 0, ctypes.byref(n), 0) == -5           # FV_ESTATE before run
    finally:
        L.fv_ctx_destroy(h)


def test_parser():
    rules = fv.parse_program("sg(x, y) :- edge(a, x), sg(a, b), edge(b, y), x != y.  % c\n"
                             "t(x, 7, _) :- t(x, 7, _).")
    (h, body, neq), (h2, body2, _) = rules
    assert h == ("sg", [("v", 1), ("v", 3)]) or h[0] == "sg"
    assert [b[0] for b in body] == ["edge", "sg", "edge"]
    assert len(neq) == 1
    assert h2[1][1] == ("c", 7)
    # the two underscores of one rule are distinct variables
    assert body2[0][1][2] != h2[1][2]
    with pytest.raises(ValueError):
        fv.parse_program("p(x) :- .")


def test_tuning_cache_roundtrip_on_host(tmp_path):
    # without a GPU the architecture reads as "unknown"
    p = tmp_path / "tune.json"
    p.write_text('{"format": "fv-tuning-1", "entries": {"unknown/sg": {"radix_bits": 11, "fuse_dedup": 1, '
                 '"set_load": 0.5, "index_load": 0.25, "max_blocks": 4096, "ms": 3.5}}}')
    t = fv.tuning_load(str(p), "sg")
    assert t == {"radix_bits": 11, "fuse_dedup": 1, "set_load": 0.5, "index_load": 0.25, "max_blocks": 4096,
                 "index_rebuild": 0, "index_sort": 0, "lookahead": 0, "dedup_ranges": 0,
                 "block_log2": [[8, 8, 8, 8], [8, 8, 8, 8]]}
    assert fv.tuning_load(str(p), "other") is None
    assert fv.tuning_load(str(tmp_path / "missing.json"), "sg") is None


def test_library_shares_torchs_hip_runtime():
    """libfv works on torch's device memory and streams, so the process must
    hold one HIP runtime: loading the library maps no second libamdhip64."""
    import subprocess
    import sys
    code = ("from paper_2501_13051_amd import fv; fv.lib(); "
            "paths = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}; "
            "print(len(paths), sorted(paths))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[0] == "1", out.stdout


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (a C program built with the host compiler prints them)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    mirrors = {"fv_tuning": fv.Tuning, "fv_options": fv.Options, "fv_stats": fv.Stats, "fv_term": fv.Term,
               "fv_atom": fv.Atom, "fv_rule": fv.Rule, "fv_kprof": fv.KProf}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fv.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, got):
        cname, field, value = line.split()
        py = mirrors[cname]
        want = ctypes.sizeof(py) if field == "size" else getattr(py, field).offset
        assert int(value) == want, (cname, field, int(value), want)
