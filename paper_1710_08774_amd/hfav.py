"""ctypes binding of libhfav.so: argument marshalling only.

Every step of the fused and unfused paths runs in the library's HIP kernels;
this module only converts Python chain descriptions into the C descriptor,
and torch tensors (or raw device addresses) into pointers.  If libhfav.so is
missing the import fails: there is no Python or CPU fallback.

Names follow the C ABI (include/hfav.h): chain_create, plan, execute,
chain_destroy, last_error, plan_term, plan_json.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from dataclasses import dataclass, field
from typing import Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfav.so")

# ----------------------------------------------------------------- constants
OK, EINVAL, EUNSAT, EDUP, ECYCLE, EUNSUP, EALIAS, ENOPLAN, EDEVICE, ESIZE = range(10)
STATUS = {0: "OK", 1: "EINVAL", 2: "EUNSAT", 3: "EDUP", 4: "ECYCLE", 5: "EUNSUP", 6: "EALIAS",
          7: "ENOPLAN", 8: "EDEVICE", 9: "ESIZE"}
# bytes of the library's static device workspace (hfav_execute_noalloc)
STATIC_WORKSPACE_BYTES = 64 << 20
F64, F32 = 0, 1
OP = {
    "HDIFF_LAP": 1, "HDIFF_FLX": 2, "HDIFF_FLY": 3, "HDIFF_OUT": 4,
    "EULER_PRIM": 10, "EULER_SLOPE": 11, "EULER_TRACE": 12, "EULER_RIEMANN": 13,
    "EULER_FLUX": 14, "EULER_UPDATE": 15, "EULER_SMAX": 16, "EULER_DT": 17,
    "LAP7": 20, "AXPY": 21, "STAR": 22,
    "SUMSQ": 30, "SUM_I": 31, "SQRT": 32, "DIV0": 33,
}
REDUCE_NONE, REDUCE_MAX, REDUCE_SUM = 0, 1, 2
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
MODE_AUTO, MODE_FUSED, MODE_UNFUSED = 0, 1, 2
PREC_NATIVE, PREC_F32_F64ACC = 0, 1
CONFIG_DEFAULT, CONFIG_TUNED, CONFIG_MODEL, CONFIG_FORCED = 0, 1, 2, 3
FAMILY = {0: "none", 1: "hdiff", 2: "euler_x", 3: "euler_y", 4: "lap7_chain", 5: "star_chain", 6: "smax",
          7: "euler_y_batch", 8: "norm", 9: "euler_xy"}
STORAGE = {0: "full", 1: "register", 2: "inner", 3: "outer", 4: "scalar"}
MAX_RULES = 64
MAX_NESTS = 8
COST_FEATURES = 24
COST_MAX_CANDIDATES = 64


class hfav_ref(C.Structure):
    _fields_ = [("term", C.c_char_p), ("off", C.c_int * 3)]


class hfav_rule(C.Structure):
    _fields_ = [("op", C.c_int), ("n_in", C.c_int), ("in_", C.POINTER(hfav_ref)),
                ("n_out", C.c_int), ("out", C.POINTER(C.c_char_p)),
                ("n_param", C.c_int), ("param", C.POINTER(C.c_double)), ("reduce", C.c_int)]


class hfav_term_decl(C.Structure):
    _fields_ = [("name", C.c_char_p), ("rank", C.c_int)]


class hfav_chain_desc(C.Structure):
    _fields_ = [("ndim", C.c_int), ("loop_order", C.c_char_p), ("dtype", C.c_int),
                ("n_axiom", C.c_int), ("axioms", C.POINTER(hfav_term_decl)),
                ("n_goal", C.c_int), ("goals", C.POINTER(C.c_char_p)),
                ("n_rule", C.c_int), ("rules", C.POINTER(hfav_rule))]


class hfav_config(C.Structure):
    _fields_ = [("block", C.c_int), ("tile_y", C.c_int), ("seg", C.c_int), ("variant", C.c_int),
                ("xcd", C.c_int)]


class hfav_plan_opts(C.Structure):
    _fields_ = [("dims", C.c_int * 3), ("boundary", C.c_int * 3), ("mode", C.c_int),
                ("precision", C.c_int), ("config_source", C.c_int), ("forced", hfav_config)]


class hfav_plan_info(C.Structure):
    _fields_ = [("n_rules", C.c_int), ("rule_order", C.c_int * MAX_RULES), ("n_nests", C.c_int),
                ("nest_of_rule", C.c_int * MAX_RULES), ("phase_of_rule", C.c_int * MAX_RULES),
                ("family", C.c_int), ("fused", C.c_int), ("streamed_axis", C.c_int),
                ("config", hfav_config), ("config_source", C.c_int),
                ("footprint_unfused", C.c_int64), ("footprint_contracted", C.c_int64),
                ("max_window", C.c_int), ("bytes_per_cell_fused", C.c_double),
                ("bytes_per_cell_unfused", C.c_double), ("workspace_bytes", C.c_size_t),
                ("outer_of_nest", C.c_int * MAX_NESTS)]


class hfav_term_info(C.Structure):
    _fields_ = [("name", C.c_char_p), ("kind", C.c_int), ("rank", C.c_int), ("producer", C.c_int),
                ("ext_lo", C.c_int * 3), ("ext_hi", C.c_int * 3), ("storage", C.c_int),
                ("window_axis", C.c_int), ("window", C.c_int)]


class hfav_nest(C.Structure):
    _fields_ = [("rank", C.c_int), ("n_prologue", C.c_int), ("n_steady", C.c_int), ("n_epilogue", C.c_int),
                ("prologue", C.c_int * MAX_RULES), ("steady", C.c_int * MAX_RULES),
                ("epilogue", C.c_int * MAX_RULES)]


class hfav_copy_desc(C.Structure):
    _fields_ = [("pattern", C.c_int), ("bytes", C.c_int64), ("slab_bytes", C.c_int64), ("slabs", C.c_int64),
                ("row_bytes", C.c_int64), ("band_bytes", C.c_int), ("tile_rows", C.c_int), ("seg", C.c_int),
                ("access_bytes", C.c_int)]


COPY_FLAT, COPY_SEGMENTS = 0, 1


# ----------------------------------------------------------------- library
_lib = None
EXPORTS = ["hfav_chain_create", "hfav_chain_infer", "hfav_chain_alias", "hfav_plan", "hfav_execute",
           "hfav_execute_noalloc", "hfav_chain_destroy", "hfav_last_error",
           "hfav_version", "hfav_num_terms", "hfav_plan_term", "hfav_plan_json",
           "hfav_tuning_clear", "hfav_tuning_add", "hfav_tuning_size"]


def lib():
    """Load libhfav.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1710_08774_amd/build.py "
                          "(there is no fallback implementation)")
    from .build import built_id, source_hash
    built, want = built_id(LIB_PATH), source_hash()
    if built != want:
        raise ImportError(f"{LIB_PATH} was built from other sources (build id {built}, sources {want}); "
                          "rebuild it with paper_1710_08774_amd/build.py")
    L = C.CDLL(LIB_PATH)
    L.hfav_build_id.restype = C.c_char_p
    L.hfav_chain_create.argtypes = [C.POINTER(hfav_chain_desc), C.POINTER(C.c_void_p)]
    L.hfav_chain_infer.argtypes = [C.POINTER(hfav_chain_desc), C.POINTER(C.c_void_p)]
    L.hfav_chain_alias.argtypes = [C.c_void_p, C.c_char_p, C.c_char_p]
    L.hfav_plan.argtypes = [C.c_void_p, C.POINTER(hfav_plan_opts), C.POINTER(hfav_plan_info)]
    L.hfav_execute.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p,
                               C.c_void_p]
    L.hfav_execute_noalloc.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p]
    L.hfav_chain_destroy.argtypes = [C.c_void_p]
    L.hfav_chain_destroy.restype = None
    L.hfav_last_error.restype = C.c_char_p
    L.hfav_version.restype = C.c_char_p
    L.hfav_num_terms.argtypes = [C.c_void_p]
    L.hfav_plan_term.argtypes = [C.c_void_p, C.c_int, C.POINTER(hfav_term_info)]
    L.hfav_plan_json.argtypes = [C.c_void_p]
    L.hfav_plan_json.restype = C.c_char_p
    L.hfav_plan_batch.argtypes = [C.c_void_p, C.POINTER(hfav_plan_opts), C.c_int, C.POINTER(C.c_int),
                                  C.POINTER(hfav_plan_info)]
    L.hfav_batch_offset.argtypes = [C.c_void_p, C.c_int]
    L.hfav_batch_offset.restype = C.c_int64
    L.hfav_mlp_nparams.argtypes = [C.c_int, C.c_int]
    L.hfav_mlp_nparams.restype = C.c_size_t
    L.hfav_mlp_workspace_bytes.argtypes = [C.c_int, C.c_int, C.c_int]
    L.hfav_mlp_workspace_bytes.restype = C.c_size_t
    L.hfav_mlp_forward.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]
    L.hfav_mlp_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
    L.hfav_mlp_adam.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_float, C.c_float,
                                C.c_float, C.c_float, C.c_int, C.c_void_p]
    L.hfav_star_candidates.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(hfav_config), C.c_int]
    L.hfav_costmodel_features.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(hfav_config),
                                          C.POINTER(C.c_float)]
    L.hfav_costmodel_set.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
    L.hfav_costmodel_predict.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(hfav_config),
                                         C.POINTER(C.c_float)]
    L.hfav_fuse_nests.argtypes = [C.c_int, C.POINTER(C.c_ubyte), C.c_int, C.POINTER(hfav_nest),
                                  C.POINTER(hfav_nest), C.POINTER(C.c_int)]
    L.hfav_copy_probe.argtypes = [C.POINTER(hfav_copy_desc), C.c_void_p, C.c_void_p, C.c_void_p]
    L.hfav_tuning_clear.restype = None
    L.hfav_tuning_add.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(hfav_config)]
    _lib = L
    return L


def last_error() -> str:
    return lib().hfav_last_error().decode()


def version() -> str:
    return lib().hfav_version().decode()


class HfavError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise HfavError(rc, last_error())


# ----------------------------------------------------------------- chain spec
@dataclass
class Rule:
    op: str
    inputs: Sequence           # (term, (di, dj, dk)) pairs
    outputs: Sequence[str]
    params: Sequence[float] = ()
    reduce: int = REDUCE_NONE


@dataclass
class ChainSpec:
    ndim: int
    axioms: Sequence           # (name, rank) pairs
    goals: Sequence[str]
    rules: Sequence[Rule]
    dtype: int = F64
    loop_order: str | None = None
    _keep: list = field(default_factory=list, repr=False)

    def to_c(self):
        keep = []
        axs = (hfav_term_decl * len(self.axioms))(*[hfav_term_decl(n.encode(), r) for n, r in self.axioms])
        goals = (C.c_char_p * len(self.goals))(*[g.encode() for g in self.goals])
        crules = (hfav_rule * max(1, len(self.rules)))()
        for q, r in enumerate(self.rules):
            refs = (hfav_ref * len(r.inputs))()
            for m, (t, off) in enumerate(r.inputs):
                o = tuple(off) + (0,) * (3 - len(off))
                refs[m] = hfav_ref(t.encode(), (C.c_int * 3)(*o))
            outs = (C.c_char_p * len(r.outputs))(*[o.encode() for o in r.outputs])
            params = (C.c_double * max(1, len(r.params)))(*[float(p) for p in r.params])
            crules[q] = hfav_rule(OP[r.op] if isinstance(r.op, str) else int(r.op), len(r.inputs), refs,
                                  len(r.outputs), outs, len(r.params), params, int(r.reduce))
            keep += [refs, outs, params]
        d = hfav_chain_desc(self.ndim, self.loop_order.encode() if self.loop_order else None, self.dtype,
                            len(self.axioms), axs, len(self.goals), goals, len(self.rules), crules)
        keep += [axs, goals, crules]
        return d, keep


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


class BoundExecute:
    """hfav_execute with buffers checked once (Chain.bind)."""

    def __init__(self, chain, axioms, goals, workspace):
        self._chain = chain
        self._gen = chain._plan_gen
        self._keep = (list(axioms), list(goals), workspace)
        self._ax = (C.c_void_p * len(axioms))(*[_ptr(a) for a in axioms])
        self._go = (C.c_void_p * len(goals))(*[_ptr(g) for g in goals])
        self._ws = _ptr(workspace)
        self._fn = lib().hfav_execute

    def stale(self):
        """True once the chain has been planned again."""
        return self._chain._plan_gen != self._gen

    def __call__(self, stream=None):
        if self._chain._plan_gen != self._gen:
            raise HfavError(ENOPLAN, "the chain was planned again after bind()")
        if stream is None:
            import torch
            s = torch.cuda.current_stream().cuda_stream
        else:
            s = stream if isinstance(stream, int) else stream.cuda_stream
        rc = self._fn(self._chain._h, self._ax, self._go, self._ws, s)
        if rc != OK:
            raise HfavError(rc, last_error())


class Chain:
    """A created chain handle (hfav_chain_create) with plan and execute."""

    def __init__(self, spec: ChainSpec, infer: bool = False):
        """infer=True: the spec's rules are patterns (hfav_chain_infer)."""
        self.spec = spec
        d, keep = spec.to_c()
        h = C.c_void_p()
        create = lib().hfav_chain_infer if infer else lib().hfav_chain_create
        _check(create(C.byref(d), C.byref(h)))
        self._h = h
        self.info = None
        self._plan_gen = 0          # bumped by every (re)plan: bound executes check it

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hfav_chain_destroy(h)
            self._h = None

    def alias(self, goal: str, axiom: str):
        """Declare an in-place pair: `goal` is written over `axiom`."""
        self._plan_gen += 1
        _check(lib().hfav_chain_alias(self._h, goal.encode(), axiom.encode()))

    def plan(self, dims, boundary=(BC_PERIODIC,) * 3, mode=MODE_AUTO, precision=PREC_NATIVE,
             config_source=CONFIG_DEFAULT, forced=None) -> hfav_plan_info:
        dims = tuple(int(x) for x in dims) + (1,) * (3 - len(dims))
        bnd = tuple(boundary) + (BC_PERIODIC,) * (3 - len(boundary))
        f = hfav_config(*(tuple(forced) + (0,) * (5 - len(forced)) if forced is not None else (0,) * 5))
        o = hfav_plan_opts((C.c_int * 3)(*dims), (C.c_int * 3)(*bnd), mode, precision, config_source, f)
        info = hfav_plan_info()
        self._plan_gen += 1
        _check(lib().hfav_plan(self._h, C.byref(o), C.byref(info)))
        self.info = info
        self.dims = dims
        self._expect = self._expected_buffers(dims[0] * dims[1] * dims[2], dims[1] * dims[2], 1)
        return info

    def plan_batch(self, sizes, boundary=(BC_PERIODIC,) * 3, precision=PREC_NATIVE,
                   config_source=CONFIG_DEFAULT, forced=None) -> hfav_plan_info:
        """Plan for a batch of grids; sizes is a list of (nx, ny)."""
        flat = (C.c_int * (2 * len(sizes)))(*[int(v) for s in sizes for v in s])
        bnd = tuple(boundary) + (BC_PERIODIC,) * (3 - len(boundary))
        f = hfav_config(*(tuple(forced) + (0,) * (5 - len(forced)) if forced is not None else (0,) * 5))
        o = hfav_plan_opts((C.c_int * 3)(1, 1, 1), (C.c_int * 3)(*bnd), MODE_FUSED, precision, config_source, f)
        info = hfav_plan_info()
        self._plan_gen += 1
        _check(lib().hfav_plan_batch(self._h, C.byref(o), len(sizes), flat, C.byref(info)))
        self.info = info
        self.sizes = list(sizes)
        total = self.batch_offset(len(sizes) - 1) + int(sizes[-1][0]) * int(sizes[-1][1])
        self._expect = self._expected_buffers(total, None, len(sizes))
        return info

    def _expected_buffers(self, n_grid, n_row, n_scalar):
        """(torch dtype, elements) the plan reads or writes through each axiom
        and goal pointer, in declaration order."""
        import torch
        grid_dt = torch.float64 if self.spec.dtype == F64 else torch.float32
        ranks = {t["name"]: t["rank"] for t in self.terms().values()}
        nd = self.spec.ndim

        def one(name):
            r = ranks[name]
            if r == 0:
                return torch.float64, n_scalar
            return grid_dt, n_grid if r == nd else n_row

        return ([one(n) for n, _ in self.spec.axioms], [one(g) for g in self.spec.goals])

    def _validate(self, axioms, goals, workspace):
        """Each tensor argument must be a contiguous device tensor of the
        plan's element type holding at least the elements the kernels touch
        (raw integer addresses are passed through unchecked)."""
        if self.info is None:
            raise HfavError(ENOPLAN, "execute before plan")
        ex_ax, ex_go = self._expect
        if len(axioms) != len(ex_ax) or len(goals) != len(ex_go):
            raise HfavError(EINVAL, f"expected {len(ex_ax)} axioms and {len(ex_go)} goals, "
                                    f"got {len(axioms)} and {len(goals)}")
        for kind, ts, ex in (("axiom", axioms, ex_ax), ("goal", goals, ex_go)):
            for q, (t, (dt, n)) in enumerate(zip(ts, ex)):
                if t is None or isinstance(t, int):
                    continue
                if t.device.type != "cuda" or not t.is_contiguous() or t.dtype != dt or t.numel() < n:
                    raise HfavError(EINVAL, f"{kind} {q}: need a contiguous cuda tensor of {dt} with >= {n} "
                                            f"elements, got {t.dtype} {tuple(t.shape)} on {t.device}"
                                            f"{'' if t.is_contiguous() else ' (not contiguous)'}")
        need = self.info.workspace_bytes
        if need and workspace is not None and not isinstance(workspace, int):
            if workspace.device.type != "cuda" or workspace.numel() * workspace.element_size() < need:
                raise HfavError(EINVAL, f"workspace: need a cuda buffer of >= {need} bytes")

    def batch_offset(self, g) -> int:
        return int(lib().hfav_batch_offset(self._h, g))

    def execute(self, axioms, goals, workspace=None, stream=None):
        """Enqueue on `stream` (torch.cuda.Stream, raw handle, or None = current)."""
        self._validate(axioms, goals, workspace)
        ax = (C.c_void_p * len(axioms))(*[_ptr(a) for a in axioms])
        go = (C.c_void_p * len(goals))(*[_ptr(g) for g in goals])
        if stream is None:
            import torch
            s = torch.cuda.current_stream().cuda_stream
        elif isinstance(stream, int):
            s = stream
        else:
            s = stream.cuda_stream
        _check(lib().hfav_execute(self._h, ax, go, _ptr(workspace), s))

    def bind(self, axioms, goals, workspace=None):
        """Validate the buffers once and return a callable that enqueues this
        execute with them (`call(stream=None)`): the per-call host work of a
        time-stepping loop is then one C call.  The binding holds the
        tensors; it refuses to run after the chain is planned again."""
        self._validate(axioms, goals, workspace)
        return BoundExecute(self, axioms, goals, workspace)

    def execute_noalloc(self, axioms, goals, stream=None):
        """hfav_execute_noalloc: the workspace is the library's static device
        array (calls on one device must not overlap)."""
        self._validate(axioms, goals, None)
        ax = (C.c_void_p * len(axioms))(*[_ptr(a) for a in axioms])
        go = (C.c_void_p * len(goals))(*[_ptr(g) for g in goals])
        if stream is None:
            import torch
            s = torch.cuda.current_stream().cuda_stream
        elif isinstance(stream, int):
            s = stream
        else:
            s = stream.cuda_stream
        _check(lib().hfav_execute_noalloc(self._h, ax, go, s))

    def execute_noalloc_status(self, axioms, goals, stream=0):
        """Like execute_noalloc but returns the status code instead of raising."""
        ax = (C.c_void_p * len(axioms))(*[_ptr(a) for a in axioms])
        go = (C.c_void_p * len(goals))(*[_ptr(g) for g in goals])
        return lib().hfav_execute_noalloc(self._h, ax, go, stream)

    def execute_status(self, axioms, goals, workspace=None, stream=0):
        """Like execute but returns the status code instead of raising."""
        ax = (C.c_void_p * len(axioms))(*[_ptr(a) for a in axioms])
        go = (C.c_void_p * len(goals))(*[_ptr(g) for g in goals])
        return lib().hfav_execute(self._h, ax, go, _ptr(workspace), stream)

    def candidates(self, dims):
        """Feasible fused configurations of a linear star chain (host)."""
        d = (C.c_int * 3)(*(tuple(dims) + (1,) * (3 - len(dims))))
        out = (hfav_config * COST_MAX_CANDIDATES)()
        n = lib().hfav_star_candidates(self._h, d, out, COST_MAX_CANDIDATES)
        if n < 0:
            raise HfavError(EUNSUP, "not a chain of linear star stages")
        return [(c.block, c.tile_y, c.seg, c.variant, c.xcd) for c in out[:n]]

    def features(self, dims, cfg):
        d = (C.c_int * 3)(*(tuple(dims) + (1,) * (3 - len(dims))))
        c = hfav_config(*(tuple(cfg) + (0,) * (5 - len(cfg))))
        f = (C.c_float * COST_FEATURES)()
        _check(lib().hfav_costmodel_features(self._h, d, C.byref(c), f))
        return list(f)

    def predict(self, dims, cfg):
        d = (C.c_int * 3)(*(tuple(dims) + (1,) * (3 - len(dims))))
        c = hfav_config(*(tuple(cfg) + (0,) * (5 - len(cfg))))
        y = C.c_float()
        _check(lib().hfav_costmodel_predict(self._h, d, C.byref(c), C.byref(y)))
        return y.value

    def num_terms(self):
        return lib().hfav_num_terms(self._h)

    def term(self, index) -> dict:
        ti = hfav_term_info()
        _check(lib().hfav_plan_term(self._h, index, C.byref(ti)))
        return {"name": ti.name.decode(), "kind": ti.kind, "rank": ti.rank, "producer": ti.producer,
                "lo": tuple(ti.ext_lo), "hi": tuple(ti.ext_hi), "storage": STORAGE[ti.storage],
                "window_axis": ti.window_axis, "window": ti.window}

    def terms(self) -> dict:
        return {t["name"]: t for t in (self.term(q) for q in range(self.num_terms()))}

    def plan_json(self) -> dict:
        s = lib().hfav_plan_json(self._h)
        if s is None:
            raise HfavError(ENOPLAN, last_error())
        return json.loads(s.decode())


def chain_create(spec: ChainSpec) -> Chain:
    return Chain(spec)


def chain_infer(spec: ChainSpec) -> Chain:
    """Chain inferred from rule patterns (pattern variables "q?")."""
    return Chain(spec, infer=True)


def fuse_nests(n_rules, reach, nests):
    """The planner's nest-fusion walk (hfav_fuse_nests) on explicit nests.

    reach: n_rules x n_rules booleans, reach[a][b] true when rule b depends on
    rule a.  nests: sequence of (rank, prologue, steady, epilogue) with rule
    ids.  Returns the fused nests in the same form."""
    flat = (C.c_ubyte * (n_rules * n_rules))(*[1 if reach[a][b] else 0 for a in range(n_rules)
                                                for b in range(n_rules)])
    src = (hfav_nest * max(1, len(nests)))()
    for q, (rank, pro, ste, epi) in enumerate(nests):
        n = src[q]
        n.rank = rank
        n.n_prologue, n.n_steady, n.n_epilogue = len(pro), len(ste), len(epi)
        for k, r in enumerate(pro):
            n.prologue[k] = r
        for k, r in enumerate(ste):
            n.steady[k] = r
        for k, r in enumerate(epi):
            n.epilogue[k] = r
    out = (hfav_nest * max(1, len(nests)))()
    n_out = C.c_int()
    _check(lib().hfav_fuse_nests(n_rules, flat, len(nests), src, out, C.byref(n_out)))
    return [(o.rank, list(o.prologue[:o.n_prologue]), list(o.steady[:o.n_steady]),
             list(o.epilogue[:o.n_epilogue])) for o in out[:n_out.value]]


def copy_probe(src, dst, pattern=COPY_FLAT, nbytes=0, slab_bytes=0, slabs=0, row_bytes=0, band_bytes=0,
               tile_rows=1, seg=1, access_bytes=8, stream=None):
    """Streaming-ceiling copy of src into dst (hfav_copy_probe)."""
    d = hfav_copy_desc(pattern, nbytes, slab_bytes, slabs, row_bytes, band_bytes, tile_rows, seg, access_bytes)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    _check(lib().hfav_copy_probe(C.byref(d), _ptr(src), _ptr(dst), stream))


def tuning_clear():
    lib().hfav_tuning_clear()


def tuning_add(family, dtype, dims, cfg):
    d = (C.c_int * 3)(*(tuple(dims) + (1,) * (3 - len(dims))))
    c = hfav_config(*(tuple(cfg) + (0,) * (5 - len(cfg))))
    _check(lib().hfav_tuning_add(int(family), int(dtype), d, C.byref(c)))


def tuning_size():
    return lib().hfav_tuning_size()


# ----------------------------------------------------------------- cost model
def mlp_nparams(d, H=64):
    return int(lib().hfav_mlp_nparams(d, H))


def mlp_workspace_bytes(n, d, H=64):
    return int(lib().hfav_mlp_workspace_bytes(n, d, H))


def _mlp_rc(rc):
    if rc != 0:
        raise HfavError(EDEVICE if rc == 8 else EINVAL, "MLP kernel call failed")


def mlp_forward(X, params, y, ws, H=64, stream=0):
    n, d = X.shape
    _mlp_rc(lib().hfav_mlp_forward(_ptr(X), n, d, H, _ptr(params), _ptr(y), _ptr(ws), stream))


def mlp_loss_grad(X, t, params, grads, loss, ws, H=64, stream=0):
    n, d = X.shape
    _mlp_rc(lib().hfav_mlp_loss_grad(_ptr(X), _ptr(t), n, d, H, _ptr(params), _ptr(grads), _ptr(loss),
                                     _ptr(ws), stream))


def mlp_adam(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=0):
    _mlp_rc(lib().hfav_mlp_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(), lr, b1, b2, eps,
                                step, stream))


def costmodel_set(params, H, mean, std):
    """Install trained weights (host sequences of floats); params=None removes."""
    if params is None:
        _check(lib().hfav_costmodel_set(None, 0, None, None))
        return
    P = (C.c_float * len(params))(*[float(x) for x in params])
    M = (C.c_float * COST_FEATURES)(*[float(x) for x in mean])
    S = (C.c_float * COST_FEATURES)(*[float(x) for x in std])
    _check(lib().hfav_costmodel_set(P, H, M, S))


# ----------------------------------------------------------------- workload chains
def hdiff_spec(coeff=0.025, dtype=F64, loop_order=None) -> ChainSpec:
    """COSMO horizontal diffusion (Performance, "COSMO Micro-Kernels")."""
    z = (0, 0, 0)
    return ChainSpec(
        ndim=3, dtype=dtype, loop_order=loop_order, axioms=[("u", 3)], goals=["out"],
        rules=[
            Rule("HDIFF_LAP", [("u", z), ("u", (1, 0, 0)), ("u", (-1, 0, 0)), ("u", (0, 1, 0)),
                               ("u", (0, -1, 0))], ["lap"]),
            Rule("HDIFF_FLX", [("lap", z), ("lap", (1, 0, 0)), ("u", z), ("u", (1, 0, 0))], ["flx"]),
            Rule("HDIFF_FLY", [("lap", z), ("lap", (0, 1, 0)), ("u", z), ("u", (0, 1, 0))], ["fly"]),
            Rule("HDIFF_OUT", [("u", z), ("flx", z), ("flx", (-1, 0, 0)), ("fly", z), ("fly", (0, -1, 0))],
                 ["out"], [coeff]),
        ])


EULER_AXIOMS = ("rho", "mx", "my", "E")
EULER_GOALS = ("rho_n", "mx_n", "my_n", "E_n")


def euler_sweep_spec(direction, gamma=1.4, niter=10, cfl=0.5, dt_source="smax", with_smax=False,
                     dtype=F64) -> ChainSpec:
    """One directional Godunov sweep (Performance, "Hydro2D").

    direction 0 sweeps x (normal momentum mx), 1 sweeps y (normal momentum my).
    dt_source "smax": a 0-D axiom `smax` and a 0-D rule dt = cfl/smax;
    "dt": a 0-D axiom `dt`.  with_smax adds the CFL reduction of the updated
    state as a 0-D goal `smax_n`.
    """
    e = (1, 0, 0) if direction == 0 else (0, 1, 0)
    me = tuple(-x for x in e)
    z = (0, 0, 0)
    rho, mx, my, E = EULER_AXIOMS
    mn, mt = (mx, my) if direction == 0 else (my, mx)
    gmn, gmt = ("mx_n", "my_n") if direction == 0 else ("my_n", "mx_n")
    prim = ["w_r", "w_un", "w_ut", "w_p", "w_c"]
    slopes = ["d_r", "d_un", "d_ut", "d_p"]
    plus = ["fp_r", "fp_un", "fp_ut", "fp_p"]
    minus = ["fm_r", "fm_un", "fm_ut", "fm_p"]
    gst = ["g_r", "g_un", "g_ut", "g_p"]
    flx = ["F_r", "F_mn", "F_mt", "F_E"]
    rules = []
    axioms = [(rho, 2), (mx, 2), (my, 2), (E, 2)]
    if dt_source == "smax":
        axioms.append(("smax", 0))
        rules.append(Rule("EULER_DT", [("smax", z)], ["dt"], [cfl]))
    else:
        axioms.append(("dt", 0))
    rules += [
        Rule("EULER_PRIM", [(rho, z), (mn, z), (mt, z), (E, z)], prim, [gamma]),
        Rule("EULER_SLOPE", [(w, o) for w in prim[:4] for o in (me, z, e)], slopes),
        Rule("EULER_TRACE", [(w, z) for w in prim] + [(d, z) for d in slopes] + [("dt", z)], plus + minus),
        Rule("EULER_RIEMANN", [(w, z) for w in plus] + [(w, e) for w in minus], gst, [gamma, niter]),
        Rule("EULER_FLUX", [(w, z) for w in gst], flx, [gamma]),
        Rule("EULER_UPDATE", [(rho, z), (mn, z), (mt, z), (E, z)] + [(f, z) for f in flx] +
             [(f, me) for f in flx] + [("dt", z)], ["rho_n", gmn, gmt, "E_n"]),
    ]
    goals = list(EULER_GOALS)
    if with_smax:
        rules.append(Rule("EULER_SMAX", [("rho_n", z), ("mx_n", z), ("my_n", z), ("E_n", z)], ["smax_n"],
                          [gamma], REDUCE_MAX))
        goals.append("smax_n")
    return ChainSpec(ndim=2, dtype=dtype, axioms=axioms, goals=goals, rules=rules)


def euler_step_spec(gamma=1.4, niter=10, cfl=0.5, dt_source="smax", with_smax=False, dtype=F64) -> ChainSpec:
    """One time step as ONE chain: the x sweep of (rho, mx, my, E) and the y
    sweep of its result with the same dt; the x-swept state is an
    intermediate (names suffixed _x), the goals are the new state.  The
    planner fuses the two equal-rank nests (Design, "Fusing iteration
    nests")."""
    xs = euler_sweep_spec(0, gamma, niter, cfl, dt_source, False, dtype)
    ys = euler_sweep_spec(1, gamma, niter, cfl, dt_source, with_smax, dtype)
    ren_x = {g: g.replace("_n", "_x") for g in EULER_GOALS}
    rules = []
    for r in xs.rules:
        outs = [ren_x.get(o, o if o == "dt" else o + "_x") for o in r.outputs]
        ins = [(t if t in EULER_AXIOMS or t in ("dt", "smax") else ren_x.get(t, t + "_x"), off)
               for t, off in r.inputs]
        rules.append(Rule(r.op, ins, outs, r.params, r.reduce))
    src = {a: ren_x[g] for a, g in zip(EULER_AXIOMS, EULER_GOALS)}      # rho -> rho_x, ...
    for r in ys.rules:
        if r.op == "EULER_DT":
            continue                                                     # dt is shared
        outs = [o if o in EULER_GOALS or o == "smax_n" else o + "_y" for o in r.outputs]
        ins = [(src[t] if t in EULER_AXIOMS else t if t in ("dt",) or t in EULER_GOALS else t + "_y", off)
               for t, off in r.inputs]
        rules.append(Rule(r.op, ins, outs, r.params, r.reduce))
    return ChainSpec(ndim=2, dtype=dtype, axioms=xs.axioms, goals=list(ys.goals), rules=rules)


def smax_spec(gamma=1.4, dtype=F64) -> ChainSpec:
    """The CFL reduction alone (initial time step)."""
    z = (0, 0, 0)
    return ChainSpec(ndim=2, dtype=dtype, axioms=[(a, 2) for a in EULER_AXIOMS], goals=["smax"],
                     rules=[Rule("EULER_SMAX", [(a, z) for a in EULER_AXIOMS], ["smax"], [gamma], REDUCE_MAX)])


def lap7_refs(t):
    return [(t, (0, 0, 0)), (t, (1, 0, 0)), (t, (-1, 0, 0)), (t, (0, 1, 0)), (t, (0, -1, 0)),
            (t, (0, 0, 1)), (t, (0, 0, -1))]


def biharm_spec(nu=1.0 / 128.0, dtype=F64) -> ChainSpec:
    """lap1 = L7(u), lap2 = L7(lap1), out = u - nu*lap2 on a 3-D box."""
    return ChainSpec(ndim=3, dtype=dtype, axioms=[("u", 3)], goals=["out"],
                     rules=[Rule("LAP7", lap7_refs("u"), ["lap1"]),
                            Rule("LAP7", lap7_refs("lap1"), ["lap2"]),
                            Rule("AXPY", [("u", (0, 0, 0)), ("lap2", (0, 0, 0))], ["out"], [-nu])])


def norm_spec(nq=4, c=1.0, dtype=F64, ndim=2, with_norm=False, loop_order=None) -> ChainSpec:
    """Normalisation chain (Performance, "Normalization Example") over nq
    fields u0..u{nq-1}: flux f_q = u_q(i+1) - u_q(i), e = sum_q f_q^2,
    s = row sum of e (a reduction along i to a row term), n = sqrt(s),
    d_q = f_q / n (0 where n = 0; a broadcast of n along i) and
    out_q = u_q - c d_q.  with_norm adds the row norm n as a goal."""
    z = (0, 0, 0)
    us = [f"u{q}" for q in range(nq)]
    rules = [Rule("STAR", [(u, (1, 0, 0)), (u, z)], [f"f{q}"], [1.0, -1.0]) for q, u in enumerate(us)]
    rules += [Rule("SUMSQ", [(f"f{q}", z) for q in range(nq)], ["e"]),
              Rule("SUM_I", [("e", z)], ["s"], reduce=REDUCE_SUM),
              Rule("SQRT", [("s", z)], ["n"])]
    rules += [Rule("DIV0", [(f"f{q}", z), ("n", z)], [f"d{q}"]) for q in range(nq)]
    rules += [Rule("AXPY", [(u, z), (f"d{q}", z)], [f"out{q}"], [-c]) for q, u in enumerate(us)]
    goals = [f"out{q}" for q in range(nq)] + (["n"] if with_norm else [])
    return ChainSpec(ndim=ndim, dtype=dtype, loop_order=loop_order, axioms=[(u, ndim) for u in us],
                     goals=goals, rules=rules)


def star_chain_spec(chain: dict, offsets_fn) -> ChainSpec:
    """Random linear star chain (dict from inputs.random_chain) as STAR rules."""
    nd = chain["ndim"]
    dtype = F64 if chain["dtype"] == "f64" else F32
    stages = chain["stages"]
    names = [[f"x{f}" for f in range(chain["n_in"])]]
    rules = []
    for s, st in enumerate(stages):
        offs = offsets_fn(nd, st["r"])
        outs = [f"s{s}_{o}" if s + 1 < len(stages) else f"y{o}" for o in range(st["f_out"])]
        for o in range(st["f_out"]):
            refs, params = [], []
            for f in range(st["f_in"]):
                for q, off in enumerate(offs):
                    refs.append((names[-1][f], off))
                    params.append(float(st["coeff"][o, f, q]))
            rules.append(Rule("STAR", refs, [outs[o]], params))
        names.append(outs)
    return ChainSpec(ndim=nd, dtype=dtype, axioms=[(n, nd) for n in names[0]], goals=names[-1], rules=rules)
