"""ctypes binding of libfv.so (include/fv.h), argument marshalling only.

Every step of the evaluation runs in the library's HIP kernels; this module
converts Python values to the C structs of the ABI, hands torch's caching
allocator and current stream to the library (PyTorch serves only as device
memory and stream plumbing), and turns error codes into exceptions.  If
libfv.so has not been built the import of the library raises: there is no
fallback evaluator here.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfv.so")

FV_OK = 0
STATUS = {0: "FV_OK", -1: "FV_EINVAL", -2: "FV_ENOMEM", -3: "FV_EARITY", -4: "FV_EUNSAFE",
          -5: "FV_ESTATE", -6: "FV_EHIP", -7: "FV_ERESERVED", -8: "FV_ETRUNC", -9: "FV_ENOTSUP"}
FV_PLAIN = 0
FV_LEARNED = 2
FV_TRACE = 4
FV_GRAPH = 8
FV_LOG_JOINS = 16
FV_HOST = 32
TRACE_COLS = 10

EXPORTED = ("fv_ctx_create", "fv_ctx_destroy", "fv_last_error", "fv_relation_create", "fv_relation_find",
            "fv_load_columns", "fv_add_rule", "fv_run_fixpoint", "fv_relation_size", "fv_export",
            "fv_delta_sizes", "fv_profile", "fv_run_batch", "fv_autotune", "fv_tuning_load",
            "fv_global_error", "fv_mlp_grad", "fv_mlp_train", "fv_mlp_predict", "fv_join_trace",
            "fv_hll_ndv", "fv_hll_ndv_noalloc")

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Tuning(ctypes.Structure):
    _fields_ = [("radix_bits", ctypes.c_uint32), ("fuse_dedup", ctypes.c_uint32), ("set_load", ctypes.c_float),
                ("index_load", ctypes.c_float), ("max_blocks", ctypes.c_uint32), ("index_rebuild", ctypes.c_uint32),
                ("index_sort", ctypes.c_uint32), ("lookahead", ctypes.c_uint32), ("dedup_ranges", ctypes.c_uint32),
                ("block_log2", (ctypes.c_uint8 * 4) * 2)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["block_log2"] = [list(row) for row in self.block_log2]
        return d


def _tuning_from_dict(d: dict) -> Tuning:
    d = dict(d)
    blocks = d.pop("block_log2", None)
    t = Tuning(**d)
    if blocks is not None:
        for c in range(2):
            for b in range(4):
                t.block_log2[c][b] = int(blocks[c][b])
    return t


class Options(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("user", ctypes.c_void_p), ("flags", ctypes.c_uint32), ("tuning", ctypes.POINTER(Tuning)),
                ("predictor", ctypes.POINTER(ctypes.c_float)), ("trace_only", ctypes.c_char_p)]


class Term(ctypes.Structure):
    _fields_ = [("value", ctypes.c_uint32), ("is_const", ctypes.c_uint32)]


class Atom(ctypes.Structure):
    _fields_ = [("rel", ctypes.c_uint32), ("arity", ctypes.c_uint32), ("terms", ctypes.POINTER(Term))]


class Rule(ctypes.Structure):
    _fields_ = [("head", Atom), ("body", ctypes.POINTER(Atom)), ("n_body", ctypes.c_uint32),
                ("neq", ctypes.POINTER(ctypes.c_uint32)), ("n_neq", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_uint32), ("redo_rounds", ctypes.c_uint32),
                ("derived_tuples", ctypes.c_uint64), ("join_output_tuples", ctypes.c_uint64),
                ("ms_total", ctypes.c_double), ("graph_captures", ctypes.c_uint32),
                ("graph_replays", ctypes.c_uint32), ("overflows", ctypes.c_uint32),
                ("predicted_joins", ctypes.c_uint32), ("qerror_median", ctypes.c_double),
                ("qerror_max", ctypes.c_double), ("reordered_rounds", ctypes.c_uint32)]


class KProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("ms", ctypes.c_double),
                ("algo_bytes", ctypes.c_double), ("items", ctypes.c_uint64)]


MAKE_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_lib = None
_streams = {}


def _engine_stream(torch, device):
    """One default-priority stream per device, reused by every Engine."""
    if device not in _streams:
        _streams[device] = torch.cuda.Stream(device=device)
    return _streams[device]


def lib():
    """Load libfv.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with __graft_entry__.build() "
                               "or python -m paper_2501_13051_amd.build")
        # torch first: its bundled HIP runtime carries the same soname as the
        # one libfv links against, so loading torch before libfv makes libfv
        # bind to torch's runtime.  Loaded the other way round the process
        # would hold two HIP runtimes, and the device memory and streams torch
        # hands over would belong to the other one.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.fv_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Options)]
        L.fv_ctx_destroy.argtypes = [vp]
        L.fv_ctx_destroy.restype = None
        L.fv_last_error.argtypes = [vp]
        L.fv_last_error.restype = ctypes.c_char_p
        L.fv_relation_create.argtypes = [vp, ctypes.c_char_p, u32, ctypes.POINTER(u32)]
        L.fv_relation_find.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(u32)]
        L.fv_load_columns.argtypes = [vp, u32, ctypes.POINTER(vp), u64, ctypes.c_int]
        L.fv_add_rule.argtypes = [vp, ctypes.POINTER(Rule)]
        L.fv_run_fixpoint.argtypes = [vp, ctypes.POINTER(Stats)]
        L.fv_relation_size.argtypes = [vp, u32, ctypes.POINTER(u64)]
        L.fv_export.argtypes = [vp, u32, ctypes.POINTER(vp), u64, ctypes.POINTER(u64), ctypes.c_int]
        L.fv_delta_sizes.argtypes = [vp, ctypes.POINTER(u64), u32, ctypes.POINTER(u32)]
        L.fv_profile.argtypes = [vp, ctypes.POINTER(KProf), u32, ctypes.POINTER(u32)]
        L.fv_run_batch.argtypes = [ctypes.POINTER(vp), u32, ctypes.POINTER(Stats)]
        L.fv_autotune.argtypes = [MAKE_FN, vp, ctypes.POINTER(Options), u32, ctypes.c_char_p, ctypes.c_char_p,
                                  ctypes.POINTER(Tuning)]
        L.fv_tuning_load.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(Tuning)]
        L.fv_global_error.argtypes = []
        L.fv_global_error.restype = ctypes.c_char_p
        opt = ctypes.POINTER(Options)
        L.fv_mlp_grad.argtypes = [opt, vp, vp, u32, vp, vp, vp]
        L.fv_mlp_train.argtypes = [opt, vp, vp, u32, u32, ctypes.c_float, u64, ctypes.c_int, vp, vp]
        L.fv_mlp_predict.argtypes = [opt, vp, u32, vp, vp]
        L.fv_hll_ndv.argtypes = [opt, ctypes.POINTER(vp), u32, u64, ctypes.c_int, vp]
        L.fv_hll_ndv_noalloc.argtypes = [ctypes.POINTER(vp), u32, u64, vp, vp]
        L.fv_join_trace.argtypes = [vp, vp, u32, ctypes.POINTER(u32)]
        for name in EXPORTED:
            if name not in ("fv_ctx_destroy", "fv_last_error", "fv_global_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


class FvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


# ------------------------------------------------------------------ program text
_TOKEN = re.compile(r"\s*(?:(:-)|(!=)|([A-Za-z_][A-Za-z0-9_]*)|(\d+)|([(),.])|(%[^\n]*))")


def parse_program(text: str):
    """Parse `head(t, ..) :- atom(t, ..), ..., x != y.` rules.

    Returns a list of (head, body, neq): head/body atoms are (name, terms)
    with terms ('v', index) or ('c', value); neq lists pairs of variable
    indices.  `_` is a fresh variable at each occurrence; `%` comments."""
    toks, pos = [], 0
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            if text[pos:].strip() == "":
                break
            raise ValueError(f"cannot parse program near {text[pos:pos + 20]!r}")
        pos = m.end()
        if m.group(6):
            continue
        for g in (1, 2, 3, 4, 5):
            if m.group(g):
                toks.append((g, m.group(g)))
                break
    rules, i = [], 0

    def expect(tok):
        nonlocal i
        if i >= len(toks) or toks[i][1] != tok:
            raise ValueError(f"expected {tok!r}")
        i += 1

    while i < len(toks):
        names = {}

        def term():
            nonlocal i
            kind, val = toks[i]
            i += 1
            if kind == 4:
                v = int(val)
                if v > 0xFFFFFFFE:
                    raise ValueError("constant out of range")
                return ("c", v)
            if kind != 3:
                raise ValueError(f"bad term {val!r}")
            if val == "_":
                names[f"_#{len(names)}"] = len(names)
                return ("v", len(names) - 1)
            if val not in names:
                names[val] = len(names)
            return ("v", names[val])

        def atom():
            nonlocal i
            kind, name = toks[i]
            if kind != 3:
                raise ValueError("expected a relation name")
            i += 1
            expect("(")
            ts = [term()]
            while toks[i][1] == ",":
                i += 1
                ts.append(term())
            expect(")")
            return (name, ts)

        head = atom()
        expect(":-")
        body, neq = [], []
        while True:
            if i + 1 < len(toks) and toks[i + 1][1] == "(":
                body.append(atom())
            else:
                a = term()
                expect("!=")
                b = term()
                if a[0] != "v" or b[0] != "v":
                    raise ValueError("!= takes variables")
                neq.append((a[1], b[1]))
            if toks[i][1] == ",":
                i += 1
                continue
            expect(".")
            break
        if len(names) > 16:
            raise ValueError("a rule may use at most 16 variables")
        rules.append((head, body, neq))
    return rules


# ------------------------------------------------------------------ engine
class Engine:
    """One fixpoint context on the current CUDA/HIP device and stream."""

    def __init__(self, flags: int = FV_PLAIN, stream=None, use_torch_allocator: bool = True, tuning=None,
                 predictor=None, trace_only: str = None):
        import torch
        self._torch = torch
        L = lib()
        self._L = L
        self._host = bool(flags & FV_HOST)
        opt = Options()
        if self._host:
            # the host evaluator needs no device, stream or device allocator
            self._device, self._stream_obj = None, None
            use_torch_allocator = False
        else:
            self._device = torch.cuda.current_device()
            # a stream of its own (default priority): the engine captures its
            # recursive round as a graph, which the legacy null stream cannot do
            s = stream if stream is not None else _engine_stream(torch, self._device)
            self._stream_obj = s
            opt.stream = ctypes.c_void_p(s.cuda_stream)
        opt.flags = flags
        if tuning is not None:
            self._tuning = tuning if isinstance(tuning, Tuning) else _tuning_from_dict(tuning)
            opt.tuning = ctypes.pointer(self._tuning)
        if trace_only is not None:
            self._trace_only = trace_only.encode()
            opt.trace_only = self._trace_only
        if predictor is not None:
            self._predictor = np.ascontiguousarray(np.asarray(predictor, dtype=np.float32))
            if self._predictor.size != 4801:
                raise ValueError("predictor must hold 4801 parameters")
            opt.predictor = self._predictor.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._live = {}
        if use_torch_allocator:
            dev, handle = self._device, self._stream_obj.cuda_stream

            def _alloc(nbytes, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, handle)
                except Exception:   # out of memory: report NULL, the library returns FV_ENOMEM
                    return None

            delete = torch.cuda.caching_allocator_delete

            def _free(ptr, stream, user):
                if ptr:
                    try:
                        delete(ptr)
                    except (AttributeError, TypeError):   # interpreter shutdown: torch is gone
                        pass

            self._alloc_cb = ALLOC_FN(_alloc)
            self._free_cb = FREE_FN(_free)
            opt.dev_alloc = self._alloc_cb
            opt.dev_free = self._free_cb
        self._opt = opt
        h = ctypes.c_void_p()
        self._check(L.fv_ctx_create(ctypes.byref(h), ctypes.byref(opt)), ctx=None)
        self._h = h
        self._rels = {}

    def _check(self, rc, ctx="self"):
        if rc != FV_OK:
            msg = self._L.fv_last_error(self._h).decode() if ctx is not None else ""
            raise FvError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            self._L.fv_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # relations
    def relation(self, name: str, arity: int) -> int:
        if name in self._rels:
            return self._rels[name][0]
        out = ctypes.c_uint32()
        self._check(self._L.fv_relation_create(self._h, name.encode(), arity, ctypes.byref(out)))
        self._rels[name] = (out.value, arity)
        return out.value

    def load(self, name: str, cols):
        """Append facts: `cols` is a list of per-column arrays (numpy on the
        host, or torch uint32/int32 tensors on the device)."""
        torch = self._torch
        arity = len(cols)
        rel = self.relation(name, arity)
        n = len(cols[0])
        keep = []
        ptrs = (ctypes.c_void_p * arity)()
        on_device = isinstance(cols[0], torch.Tensor) and cols[0].is_cuda
        for c, col in enumerate(cols):
            if len(col) != n:
                raise ValueError("columns differ in length")
            if on_device:
                if c == 0 and self._stream_obj is not None:   # produced on the caller's stream
                    self._stream_obj.wait_stream(torch.cuda.current_stream())
                elif c == 0:
                    torch.cuda.current_stream().synchronize()
                t = col.contiguous()
                if t.element_size() != 4:
                    raise ValueError("device columns must be 32-bit")
                keep.append(t)
                ptrs[c] = t.data_ptr()
            else:
                a = np.ascontiguousarray(np.asarray(col), dtype=np.uint32)
                keep.append(a)
                ptrs[c] = a.ctypes.data
        self._check(self._L.fv_load_columns(self._h, rel, ptrs, n, 1 if on_device else 0))

    def add_rule(self, head, body, neq=()):
        """head/body atoms are (name, terms) with terms ('v', i) / ('c', k)."""
        keep = []

        def atom(a):
            name, ts = a
            rel = self.relation(name, len(ts)) if name not in self._rels else self._rels[name][0]
            arr = (Term * len(ts))(*[Term(v, 1 if k == "c" else 0) for k, v in ts])
            keep.append(arr)
            return Atom(rel, len(ts), arr)

        r = Rule()
        r.head = atom(head)
        bodies = (Atom * len(body))(*[atom(b) for b in body])
        r.body = bodies
        r.n_body = len(body)
        flat = [x for pair in neq for x in pair]
        na = (ctypes.c_uint32 * max(1, len(flat)))(*flat)
        r.neq = na
        r.n_neq = len(neq)
        self._check(self._L.fv_add_rule(self._h, ctypes.byref(r)))

    def program(self, text: str):
        for head, body, neq in parse_program(text):
            self.add_rule(head, body, neq)

    def run(self) -> dict:
        st = Stats()
        self._check(self._L.fv_run_fixpoint(self._h, ctypes.byref(st)))
        return _stats_dict(st)

    def size(self, name: str) -> int:
        n = ctypes.c_uint64()
        self._check(self._L.fv_relation_size(self._h, self._rels[name][0], ctypes.byref(n)))
        return n.value

    def export(self, name: str, device: bool = False):
        """Relation as a row-sorted (n, arity) uint32 numpy array, or with
        device=True as a list of torch int32 column tensors (same bits)."""
        torch = self._torch
        rel, arity = self._rels[name]
        n = ctypes.c_uint64()
        self._check(self._L.fv_export(self._h, rel, None, 0, ctypes.byref(n), 0))
        n = n.value
        ptrs = (ctypes.c_void_p * arity)()
        if device:
            cols = [torch.empty(max(n, 1), dtype=torch.int32, device=f"cuda:{self._device}") for _ in range(arity)]
            for c in range(arity):
                ptrs[c] = cols[c].data_ptr()
            self._check(self._L.fv_export(self._h, rel, ptrs, n, None, 1))
            return [c[:n] for c in cols]
        out = np.zeros((arity, max(n, 1)), dtype=np.uint32)
        for c in range(arity):
            ptrs[c] = out[c].ctypes.data
        self._check(self._L.fv_export(self._h, rel, ptrs, n, None, 0))
        return np.ascontiguousarray(out[:, :n].T)

    def join_trace(self) -> np.ndarray:
        """(n, 10) float32: 8 features, log2(1+true size)/16, predicted size or -1."""
        n = ctypes.c_uint32()
        self._check(self._L.fv_join_trace(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros((max(n.value, 1), TRACE_COLS), np.float32)
        self._check(self._L.fv_join_trace(self._h, out.ctypes.data, n.value, ctypes.byref(n)))
        return out[:n.value]

    def delta_sizes(self):
        n = ctypes.c_uint32()
        self._check(self._L.fv_delta_sizes(self._h, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_uint64 * max(1, n.value))()
        self._check(self._L.fv_delta_sizes(self._h, buf, n.value, ctypes.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    def profile(self):
        n = ctypes.c_uint32()
        self._check(self._L.fv_profile(self._h, None, 0, ctypes.byref(n)))
        buf = (KProf * max(1, n.value))()
        self._check(self._L.fv_profile(self._h, buf, n.value, ctypes.byref(n)))
        return [{"name": buf[i].name.decode(), "launches": int(buf[i].launches), "ms": float(buf[i].ms),
                 "algo_bytes": float(buf[i].algo_bytes), "items": int(buf[i].items)} for i in range(n.value)]


def _stats_dict(st) -> dict:
    return {f: getattr(st, f) for f, _ in Stats._fields_}


def run_batch(engines) -> dict:
    """Evaluate engines holding the same program as one batched fixpoint
    (fv_run_batch); afterwards each engine exports its own relations."""
    L = lib()
    arr = (ctypes.c_void_p * len(engines))(*[e._h for e in engines])
    st = Stats()
    rc = L.fv_run_batch(arr, len(engines), ctypes.byref(st))
    if rc != FV_OK:
        raise FvError(rc, L.fv_last_error(engines[0]._h).decode())
    # the merged result frees its memory through the first engine's allocator
    keep = (engines[0]._opt, getattr(engines[0], "_alloc_cb", None), getattr(engines[0], "_free_cb", None))
    for e in engines:
        e._batch_keep = keep
    return _stats_dict(st)


def autotune(make_engine, key: str = None, cache_path: str = None, reps: int = 3, flags: int = FV_PLAIN):
    """Run the library's autotuner.  make_engine(tuning) must return a fresh
    Engine (created with that tuning) holding the program and facts; the
    library runs and destroys each one.  Returns the chosen tuning as a dict."""
    L = lib()
    held, failures = [], []

    def _make(opt_ptr, user):
        try:
            opt = ctypes.cast(opt_ptr, ctypes.POINTER(Options)).contents
            t = Tuning()
            ctypes.memmove(ctypes.byref(t), opt.tuning, ctypes.sizeof(Tuning))
            e = make_engine(t)
            held.append(e)
            h = e._h
            e._h = None          # the library destroys this context
            return h.value       # a plain address: ctypes cannot return a c_void_p object
        except Exception as ex:  # a failed factory is reported as NULL; keep why
            failures.append(f"{type(ex).__name__}: {ex}")
            return None

    cb = MAKE_FN(_make)
    best = Tuning()
    rc = L.fv_autotune(cb, None, None, reps, cache_path.encode() if cache_path else None,
                       key.encode() if key else None, ctypes.byref(best))
    if rc != FV_OK:
        why = f" ({failures[-1]})" if failures else ""
        raise FvError(rc, L.fv_global_error().decode() + why)
    return best.as_dict()


MLP_PARAMS = 4801
_call_opts = {}


def _call_options():
    """fv_options for the context-free calls: the current device's engine
    stream and torch's caching allocator (kept alive per device)."""
    import torch
    dev = torch.cuda.current_device()
    if dev not in _call_opts:
        s = _engine_stream(torch, dev)
        handle = s.cuda_stream

        def _alloc(nbytes, stream, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, handle)
            except Exception:
                return None

        delete = torch.cuda.caching_allocator_delete

        def _free(ptr, stream, user):
            if ptr:
                try:
                    delete(ptr)
                except (AttributeError, TypeError):
                    pass

        o = Options()
        o.stream = ctypes.c_void_p(handle)
        a, f = ALLOC_FN(_alloc), FREE_FN(_free)
        o.dev_alloc, o.dev_free = a, f
        _call_opts[dev] = (o, a, f, s)
    return ctypes.byref(_call_opts[dev][0])


def _mlp_check(rc):
    if rc != FV_OK:
        raise FvError(rc, lib().fv_global_error().decode())


def _f32(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None:
        a = a.reshape(shape)
    return a


def mlp_grad(X, y, params):
    """(loss, gradient) of the predictor MLP on (X, y), computed on the GPU."""
    X, y, P = _f32(X, (-1, 8)), _f32(y, (-1,)), _f32(params, (MLP_PARAMS,))
    g = np.zeros(MLP_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    _mlp_check(lib().fv_mlp_grad(_call_options(), X.ctypes.data, y.ctypes.data, len(y), P.ctypes.data,
                                 g.ctypes.data, loss.ctypes.data))
    return float(loss[0]), g


def mlp_train(X, y, steps=2000, lr=1e-3, seed=1, params=None):
    """Train the predictor on the GPU; returns (params, final loss)."""
    X, y = _f32(X, (-1, 8)), _f32(y, (-1,))
    P = np.zeros(MLP_PARAMS, np.float32) if params is None else _f32(params, (MLP_PARAMS,)).copy()
    loss = np.zeros(1, np.float32)
    _mlp_check(lib().fv_mlp_train(_call_options(), X.ctypes.data, y.ctypes.data, len(y), steps, lr, seed,
                                  1 if params is None else 0, P.ctypes.data, loss.ctypes.data))
    return P, float(loss[0])


def mlp_predict(X, params):
    """BF16 inference of the predictor on the GPU."""
    X, P = _f32(X, (-1, 8)), _f32(params, (MLP_PARAMS,))
    out = np.zeros(len(X), np.float32)
    _mlp_check(lib().fv_mlp_predict(_call_options(), X.ctypes.data, len(X), P.ctypes.data, out.ctypes.data))
    return out


def hll_ndv(cols):
    """HyperLogLog distinct-value estimate of each column (numpy uint32 on
    the host, or torch 32-bit tensors on the device), one sketch per column."""
    import torch
    cols = list(cols)
    if not cols:
        return np.zeros(0)
    n = len(cols[0])
    on_device = isinstance(cols[0], torch.Tensor) and cols[0].is_cuda
    keep, ptrs = [], (ctypes.c_void_p * len(cols))()
    for c, col in enumerate(cols):
        if len(col) != n:
            raise ValueError("columns differ in length")
        if on_device:
            t = col.contiguous()
            if t.element_size() != 4:
                raise ValueError("device columns must be 32-bit")
            _engine_stream(torch, torch.cuda.current_device()).wait_stream(torch.cuda.current_stream())
            keep.append(t)
            ptrs[c] = t.data_ptr()
        else:
            a = np.ascontiguousarray(np.asarray(col), dtype=np.uint32)
            keep.append(a)
            ptrs[c] = a.ctypes.data
    out = np.zeros(len(cols), np.float64)
    _mlp_check(lib().fv_hll_ndv(_call_options(), ptrs, len(cols), n, 1 if on_device else 0, out.ctypes.data))
    return out


HLL_NOALLOC_MAX_COLS = 8


def hll_ndv_noalloc(cols, out, stream=None):
    """fv_hll_ndv_noalloc: sketch up to 8 device columns (torch 32-bit
    tensors) into `out`, a float64 device tensor of len(cols), on `stream`
    (default: the current stream).  Nothing is allocated and nothing waits."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    ptrs = (ctypes.c_void_p * max(1, len(cols)))()
    n = len(cols[0]) if cols else 0
    for c, col in enumerate(cols):
        if len(col) != n or col.element_size() != 4 or not col.is_contiguous():
            raise ValueError("columns must be contiguous 32-bit tensors of one length")
        ptrs[c] = col.data_ptr()
    if out.dtype != torch.float64 or out.numel() < len(cols):
        raise ValueError("out must be a float64 tensor with one entry per column")
    _mlp_check(lib().fv_hll_ndv_noalloc(ptrs, len(cols), n, out.data_ptr(), s.cuda_stream))


def tuning_load(cache_path: str, key: str):
    """Tuning stored by autotune for this GPU's architecture, or None."""
    t = Tuning()
    if lib().fv_tuning_load(cache_path.encode(), key.encode(), ctypes.byref(t)) != FV_OK:
        return None
    return t.as_dict()


def evaluate(program: str, edb: dict, flags: int = FV_PLAIN, relations=None, device_out: bool = False,
             tuning=None, predictor=None, with_trace: bool = False):
    """Load `edb` (name -> list of columns), run `program` to its fixpoint on
    the GPU and return (relations as row-sorted arrays, stats, delta sizes,
    kernel profile) -- plus the join trace when with_trace."""
    eng = Engine(flags=flags, tuning=tuning, predictor=predictor)
    try:
        rules = parse_program(program)
        arities = {}
        for head, body, _ in rules:
            for name, ts in [head] + body:
                arities.setdefault(name, len(ts))
        for name, cols in edb.items():
            arities.setdefault(name, len(cols))
        for name, a in arities.items():
            eng.relation(name, a)
        for name, cols in edb.items():
            eng.load(name, cols)
        for head, body, neq in rules:
            eng.add_rule(head, body, neq)
        stats = eng.run()
        names = relations if relations is not None else list(arities)
        out = {name: eng.export(name, device=device_out) for name in names}
        prof = eng.profile()
        if with_trace:
            return out, stats, eng.delta_sizes(), prof, eng.join_trace()
        return out, stats, eng.delta_sizes(), prof
    finally:
        eng.close()
