"""ctypes binding of the cwcssa C ABI (include/cwcssa.h).

Argument marshalling only: every step of the simulation runs in the
library's HIP kernels.  PyTorch supplies device memory (an optional arena
tensor, device result tensors) and streams; model dictionaries are those of
the ``workloads`` module.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libcwcssa.so")

CWC_OK = 0
ERRORS = {-1: "CWC_E_INVALID", -2: "CWC_E_UNSUPPORTED", -3: "CWC_E_NOMEM",
          -4: "CWC_E_DEVICE", -5: "CWC_E_NOTREADY", -6: "CWC_E_COMPILE"}
MODE_PLAIN, MODE_PERSISTENT = 0, 1
REGION = {"p": 0, "w": 1, "c": 2}

# exported symbols, in the order include/cwcssa.h declares them
SYMBOLS = [
    "cwc_abi_version", "cwc_last_error", "cwc_ctx_create", "cwc_ctx_destroy",
    "cwc_model_create", "cwc_model_get_info", "cwc_model_source",
    "cwc_model_destroy", "cwc_model_describe", "cwc_codegen", "cwc_gmodel_create",
    "cwc_gcodegen", "cwc_run_submit", "cwc_run_relaunch",
    "cwc_run_query", "cwc_run_wait", "cwc_run_wait_for", "cwc_run_elapsed", "cwc_run_kernel_name",
    "cwc_run_fetch_stats",
    "cwc_run_fetch_moments", "cwc_run_fetch_trajectories", "cwc_run_fetch_term",
    "cwc_run_fetch_counters", "cwc_run_destroy", "cwc_run_into",
    "cwc_stream_open", "cwc_stream_next", "cwc_stream_info", "cwc_stream_fetch_counters",
    "cwc_stream_fetch_term", "cwc_stream_destroy", "cwc_server_create", "cwc_server_set_policy",
    "cwc_server_submit", "cwc_server_poll", "cwc_server_job_info",
    "cwc_server_fetch_stats", "cwc_server_fetch_counters", "cwc_server_fetch_term",
    "cwc_server_release",
    "cwc_server_wait_idle", "cwc_server_get_stats", "cwc_server_destroy",
    "cwc_autotune",
    "cwc_realign",
    "cwc_stats_confidence",
    "cwc_stats_finalize",
]


class CwcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, str(code)), msg))
        self.code = code


class cwc_stream_info_t(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_size_t), ("window", ctypes.c_int32),
                ("n_windows", ctypes.c_int32), ("windows_done", ctypes.c_int32),
                ("last_window_ms", ctypes.c_float), ("kernel", ctypes.c_char * 48)]


class cwc_term(ctypes.Structure):
    _fields_ = [("region", ctypes.c_int32), ("species", ctypes.c_int32),
                ("mult", ctypes.c_int32)]


class cwc_rule(ctypes.Structure):
    _fields_ = [("parent_type", ctypes.c_int32), ("child_type", ctypes.c_int32),
                ("n_lhs", ctypes.c_int32), ("lhs", ctypes.POINTER(cwc_term)),
                ("n_rhs", ctypes.c_int32), ("rhs", ctypes.POINTER(cwc_term)),
                ("k", ctypes.c_double)]


class cwc_gcomp(ctypes.Structure):
    _fields_ = [("label", ctypes.c_int32), ("parent", ctypes.c_int32),
                ("wrap", ctypes.c_void_p), ("content", ctypes.c_void_p)]


class cwc_grule(ctypes.Structure):
    _fields_ = [("context", ctypes.c_int32), ("child", ctypes.c_int32),
                ("grandchild", ctypes.c_int32), ("n_lhs", ctypes.c_int32),
                ("lhs", ctypes.c_void_p), ("n_rhs", ctypes.c_int32), ("rhs", ctypes.c_void_p),
                ("action", ctypes.c_int32), ("level", ctypes.c_int32),
                ("new_label", ctypes.c_int32), ("new_wrap", ctypes.c_void_p),
                ("new_content", ctypes.c_void_p), ("release_wrap", ctypes.c_int32),
                ("k", ctypes.c_double)]


class cwc_gmodel_desc(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_labels", ctypes.c_int32),
                ("has_wrap", ctypes.c_void_p), ("max_comp", ctypes.c_int32),
                ("n_comp", ctypes.c_int32), ("comps", ctypes.c_void_p),
                ("n_rules", ctypes.c_int32), ("rules", ctypes.c_void_p)]


class cwc_model_desc(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_types", ctypes.c_int32),
                ("n_comp", ctypes.c_int32),
                ("type_has_wrap", ctypes.POINTER(ctypes.c_int32)),
                ("comp_type", ctypes.POINTER(ctypes.c_int32)),
                ("comp_parent", ctypes.POINTER(ctypes.c_int32)),
                ("init_counts", ctypes.POINTER(ctypes.c_int32)),
                ("n_rules", ctypes.c_int32), ("rules", ctypes.POINTER(cwc_rule))]


class cwc_model_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("n_cells", "n_slots", "n_leaves", "p_local", "n_rules", "layout")] + \
        [("alg_slots_per_event", ctypes.c_double)]


class cwc_tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("block_size", "waves_per_simd", "refill_chunk", "lanes_per_replica",
                 "sample_slots")]


class cwc_run_desc(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_instances", ctypes.c_int64),
                ("replicas_per_instance", ctypes.c_int64),
                ("rate_table", ctypes.c_void_p), ("init_table", ctypes.c_void_p),
                ("dt", ctypes.c_double), ("n_samples", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("want_traj", ctypes.c_int32),
                ("want_digest", ctypes.c_int32), ("count_cap", ctypes.c_int32),
                ("max_events", ctypes.c_int64),
                ("tuning", ctypes.POINTER(cwc_tuning))]


class cwc_run_outputs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("mean", "var", "n", "events", "status", "digest", "t_final", "n_recorded",
                 "final_counts")]


class cwc_job_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("n_ticks", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("events", ctypes.c_int64),
                ("bytes", ctypes.c_int64)]


class cwc_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("jobs_submitted", "jobs_done", "ticks", "events", "pool_bytes",
                 "pool_used", "pool_peak")] + [("busy_s", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libcwcssa.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("cwcssa library not built: %s missing (run "
                          "__graft_entry__.build() or paper_1010_2438_amd/build.py)" % path)
    # One HIP runtime per process: PyTorch ships its own libamdhip64 under
    # the same soname.  Loading torch first makes the library bind to that
    # copy; loading torch after the library would bring in a second runtime,
    # and the two then fail to share the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    P, I32, I64, S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.cwc_abi_version.restype = ctypes.c_uint32
    L.cwc_last_error.restype = ctypes.c_char_p
    sig = {
        "cwc_ctx_create": [ctypes.c_int, P, S, ctypes.POINTER(P)],
        "cwc_model_create": [P, ctypes.POINTER(cwc_model_desc), ctypes.POINTER(P)],
        "cwc_model_get_info": [P, ctypes.POINTER(cwc_model_info)],
        "cwc_model_source": [P, ctypes.c_char_p, S, ctypes.POINTER(S)],
        "cwc_codegen": [ctypes.POINTER(cwc_model_desc), ctypes.c_char_p, S, ctypes.POINTER(S)],
        "cwc_model_describe": [ctypes.POINTER(cwc_model_desc), ctypes.POINTER(cwc_model_info)],
        "cwc_run_submit": [P, P, ctypes.POINTER(cwc_run_desc), P, ctypes.POINTER(P)],
        "cwc_run_relaunch": [P, P],
        "cwc_run_query": [P, ctypes.POINTER(ctypes.c_int)],
        "cwc_run_wait": [P],
        "cwc_run_wait_for": [P, ctypes.c_double],
        "cwc_run_elapsed": [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
        "cwc_run_kernel_name": [P, ctypes.c_char_p, S, ctypes.POINTER(S)],
        "cwc_run_fetch_stats": [P, P, P, P, ctypes.c_int],
        "cwc_run_fetch_moments": [P, P, P, P, P, ctypes.c_int],
        "cwc_run_fetch_trajectories": [P, P, ctypes.c_int],
        "cwc_run_fetch_term": [P, P, ctypes.c_int],
        "cwc_gmodel_create": [P, ctypes.POINTER(cwc_gmodel_desc), ctypes.POINTER(P)],
        "cwc_gcodegen": [ctypes.POINTER(cwc_gmodel_desc), ctypes.c_char_p, S, ctypes.POINTER(S)],
        "cwc_run_fetch_counters": [P, P, P, P, P, P, P, ctypes.c_int],
        "cwc_run_into": [P, P, ctypes.POINTER(cwc_run_desc), ctypes.POINTER(cwc_run_outputs), P],
        "cwc_stream_open": [P, P, ctypes.POINTER(cwc_run_desc), I32, P, ctypes.POINTER(P)],
        "cwc_stream_next": [P, ctypes.POINTER(I32), ctypes.POINTER(I32), P, P, P, ctypes.c_int],
        "cwc_stream_info": [P, ctypes.POINTER(cwc_stream_info_t)],
        "cwc_stream_fetch_counters": [P, P, P, P, P, P, P, ctypes.c_int],
        "cwc_stream_fetch_term": [P, P, ctypes.c_int],
        "cwc_stats_finalize": [P, P, P, P, P, I64, I32, P, P, P],
        "cwc_stats_confidence": [P, P, I64, I32, ctypes.c_double, P],
        "cwc_realign": [P, P, I64, I32, ctypes.c_double, I32, I32, P],
        "cwc_server_create": [P, S, I32, I64, ctypes.POINTER(P)],
        "cwc_autotune": [P, P, ctypes.POINTER(cwc_run_desc), ctypes.c_double,
                         ctypes.POINTER(cwc_tuning)],
        "cwc_server_set_policy": [P, I32, I32],
        "cwc_server_submit": [P, P, ctypes.POINTER(cwc_run_desc), ctypes.POINTER(ctypes.c_uint64)],
        "cwc_server_poll": [P, P, I32, ctypes.POINTER(I32)],
        "cwc_server_job_info": [P, ctypes.c_uint64, ctypes.POINTER(cwc_job_info)],
        "cwc_server_fetch_stats": [P, ctypes.c_uint64, P, P, P, ctypes.c_int],
        "cwc_server_fetch_counters": [P, ctypes.c_uint64, P, P, P, P, P, P, ctypes.c_int],
        "cwc_server_fetch_term": [P, ctypes.c_uint64, P, ctypes.c_int],
        "cwc_server_release": [P, ctypes.c_uint64],
        "cwc_server_wait_idle": [P, ctypes.c_double],
        "cwc_server_get_stats": [P, ctypes.POINTER(cwc_server_stats)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    for name in ("cwc_ctx_destroy", "cwc_model_destroy", "cwc_run_destroy",
                 "cwc_server_destroy", "cwc_stream_destroy"):
        getattr(L, name).argtypes = [P]
        getattr(L, name).restype = None
    _lib = L
    return L


def check(code: int):
    if code != CWC_OK:
        raise CwcError(code, load().cwc_last_error().decode())


# ------------------------------------------------------------- marshalling

class _ModelDesc:
    """Keeps the ctypes arrays of a cwc_model_desc alive."""

    def __init__(self, model: Dict):
        ns = len(model["species"])
        types, comps = model["types"], model["compartments"]
        self.has_wrap = (ctypes.c_int32 * len(types))(*[int(bool(t["wrap"])) for t in types])
        self.comp_type = (ctypes.c_int32 * len(comps))(*[c["type"] for c in comps])
        self.comp_parent = (ctypes.c_int32 * len(comps))(*[c["parent"] for c in comps])
        init = []
        iw = model.get("init_wrap") or [None] * len(comps)
        for i, c in enumerate(comps):
            init.extend(int(x) for x in model["init"][i])
            if types[c["type"]]["wrap"]:
                init.extend(int(x) for x in (iw[i] if iw[i] is not None else [0] * ns))
        self.init = (ctypes.c_int32 * max(1, len(init)))(*init)
        self.terms = []
        rules = []
        for r in model["rules"]:
            sides = []
            for side in ("lhs", "rhs"):
                ts = [cwc_term(REGION[reg], int(sp), int(m))
                      for reg, atoms in r[side].items() for sp, m in atoms.items()
                      if int(m) > 0]
                arr = (cwc_term * max(1, len(ts)))(*ts)
                self.terms.append(arr)
                sides.append((len(ts), arr))
            rules.append(cwc_rule(r["parent"], r["child"], sides[0][0], sides[0][1],
                                  sides[1][0], sides[1][1], float(r["k"])))
        self.rules = (cwc_rule * max(1, len(rules)))(*rules)
        self.desc = cwc_model_desc(ns, len(types), len(comps), self.has_wrap,
                                   self.comp_type, self.comp_parent, self.init,
                                   len(rules), self.rules)


GREGION = {"c": 0, "w1": 1, "c1": 2, "w2": 3, "c2": 4}
GACTION = {"none": 0, "create": 1, "dissolve": 2, "delete": 3}


class _GModelDesc:
    """Keeps the ctypes arrays of a cwc_gmodel_desc alive (general models
    of the ``workloads`` module)."""

    def __init__(self, model: Dict):
        ns = len(model["species"])
        labels = model["labels"]
        keep = self.keep = []

        def ivec(v):
            if v is None:
                return None
            if isinstance(v, dict):
                x = [0] * ns
                for a, m in v.items():
                    x[int(a)] += int(m)
                v = x
            arr = (ctypes.c_int32 * ns)(*[int(t) for t in v])
            keep.append(arr)
            return ctypes.addressof(arr)

        self.has_wrap = (ctypes.c_int32 * len(labels))(*[int(bool(l["wrap"])) for l in labels])
        comps = [cwc_gcomp(c["label"], c["parent"], ivec(c.get("wrap")), ivec(c.get("content")))
                 for c in model["term"]]
        self.comps = (cwc_gcomp * len(comps))(*comps)
        rules = []
        for r in model["rules"]:
            sides = []
            for side in ("lhs", "rhs"):
                ts = [cwc_term(GREGION[reg], int(sp), int(m))
                      for reg, atoms in r.get(side, {}).items() for sp, m in atoms.items()
                      if int(m) > 0]
                arr = (cwc_term * max(1, len(ts)))(*ts)
                keep.append(arr)
                sides.append((len(ts), ctypes.addressof(arr)))
            nw = r.get("new") or {}
            rules.append(cwc_grule(r["context"], r.get("child", -1), r.get("grandchild", -1),
                                   sides[0][0], sides[0][1], sides[1][0], sides[1][1],
                                   GACTION[r.get("action", "none")], int(r.get("level", 0)),
                                   int(nw.get("label", -1)), ivec(nw.get("wrap")),
                                   ivec(nw.get("content")), int(bool(r.get("release_wrap"))),
                                   float(r["k"])))
        self.rules = (cwc_grule * max(1, len(rules)))(*rules)
        self.desc = cwc_gmodel_desc(ns, len(labels), ctypes.addressof(self.has_wrap),
                                    int(model["max_comp"]), len(comps),
                                    ctypes.addressof(self.comps), len(rules),
                                    ctypes.addressof(self.rules))


def gcodegen(model: Dict) -> str:
    """cwc_gcodegen: the generated device source of a general model (host only)."""
    L = load()
    md = _GModelDesc(model)
    n = ctypes.c_size_t()
    check(L.cwc_gcodegen(ctypes.byref(md.desc), None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    check(L.cwc_gcodegen(ctypes.byref(md.desc), buf, n.value, ctypes.byref(n)))
    return buf.value.decode()


def confidence(var, n, level: float = 0.9):
    """cwc_stats_confidence: half-widths of the two-sided Student-t interval
    (level 0.9: the paper's 90 % band) for variances var [..., cells] and
    counts n [...]; NaN where n < 2."""
    var = np.ascontiguousarray(var, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.int64)
    cells = var.shape[-1]
    rows = n.size
    assert var.size == rows * cells
    out = np.empty_like(var)
    check(load().cwc_stats_confidence(var.ctypes.data, n.ctypes.data, rows, cells,
                                      float(level), out.ctypes.data))
    return out


def realign(times, values, dt: float, n_samples: int, fill: int = -1):
    """cwc_realign: a trajectory recorded at `times` (non-decreasing) with
    states `values` [n][cells] onto the grid k*dt, k < n_samples
    (right-continuous); rows before the first record get `fill`."""
    times = np.ascontiguousarray(times, dtype=np.float64)
    values = np.ascontiguousarray(values, dtype=np.int32)
    n = times.shape[0]
    cells = values.shape[1] if values.ndim == 2 else 1
    assert values.size == n * cells
    out = np.empty((n_samples, cells), np.int32)
    check(load().cwc_realign(times.ctypes.data, values.ctypes.data, n, cells, float(dt),
                             int(n_samples), int(fill), out.ctypes.data))
    return out


def cwc_codegen(model: Dict) -> str:
    """Generated device source for a model (host only, no device)."""
    L = load()
    md = _ModelDesc(model)
    n = ctypes.c_size_t()
    check(L.cwc_codegen(ctypes.byref(md.desc), None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    check(L.cwc_codegen(ctypes.byref(md.desc), buf, n.value, ctypes.byref(n)))
    return buf.value.decode()


def cwc_model_describe(model: Dict) -> Dict:
    """Flattened structure of a model (host only, no device)."""
    md = _ModelDesc(model)
    info = cwc_model_info()
    check(load().cwc_model_describe(ctypes.byref(md.desc), ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in cwc_model_info._fields_}


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """cwc_ctx_create / cwc_ctx_destroy.  ``arena_bytes`` > 0 allocates a
    torch uint8 tensor on the device and hands its storage to the library
    as the arena."""

    def __init__(self, device: int = 0, arena_bytes: int = 0):
        L = load()
        self.arena = None
        ptr, nbytes = None, 0
        if arena_bytes:
            import torch
            self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda:%d" % device)
            ptr, nbytes = self.arena.data_ptr(), arena_bytes
        h = ctypes.c_void_p()
        check(L.cwc_ctx_create(device, ptr, nbytes, ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            load().cwc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """cwc_model_create from a model dictionary."""

    def __init__(self, ctx: Context, model: Dict):
        L = load()
        self.ctx = ctx
        self.dict = model
        md = _ModelDesc(model)
        h = ctypes.c_void_p()
        check(L.cwc_model_create(ctx.h, ctypes.byref(md.desc), ctypes.byref(h)))
        self.h = h
        info = cwc_model_info()
        check(L.cwc_model_get_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in cwc_model_info._fields_}

    def autotune(self, run: Dict, mode="persistent", budget_s=5.0) -> Dict:
        """cwc_autotune: fastest launch shape for this run (stored for later
        submissions of the same model/mode/size class)."""
        d, _r, _i = _run_desc(run)
        d.mode = MODE_PERSISTENT if mode == "persistent" else MODE_PLAIN
        t = cwc_tuning()
        check(load().cwc_autotune(self.ctx.h, self.h, ctypes.byref(d), float(budget_s),
                                  ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in cwc_tuning._fields_}

    def source(self) -> str:
        L = load()
        n = ctypes.c_size_t()
        check(L.cwc_model_source(self.h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        check(L.cwc_model_source(self.h, buf, n.value, ctypes.byref(n)))
        return buf.value.decode()

    def close(self):
        if getattr(self, "h", None):
            load().cwc_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GModel(Model):
    """cwc_gmodel_create from a general model dictionary (compartments
    created, dissolved and deleted at run time); runs like any Model."""

    def __init__(self, ctx: Context, model: Dict):
        L = load()
        self.ctx = ctx
        self.dict = model
        md = _GModelDesc(model)
        h = ctypes.c_void_p()
        check(L.cwc_gmodel_create(ctx.h, ctypes.byref(md.desc), ctypes.byref(h)))
        self.h = h
        info = cwc_model_info()
        check(L.cwc_model_get_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in cwc_model_info._fields_}
        self.max_comp = int(model["max_comp"])
        self.n_species = len(model["species"])


class Run:
    """cwc_run_submit and the fetches.  ``run`` is a workloads.make_run
    dictionary; ``mode`` 'plain' or 'persistent'."""

    def __init__(self, ctx: Context, model: Model, run: Dict, mode="plain",
                 want_traj=False, want_digest=False, tuning: Optional[Dict] = None,
                 stream=None):
        L = load()
        self.ctx, self.model = ctx, model
        self.I, self.R = run["n_instances"], run["replicas"]
        self.G = self.I * self.R
        self.K1 = run["n_samples"]
        self.C = model.info["n_cells"]
        self._rate = run.get("rate_table")
        self._init = run.get("init_table")
        if self._rate is not None:
            self._rate = np.ascontiguousarray(self._rate, dtype=np.float64)
            assert self._rate.shape == (self.I, model.info["n_rules"])
        if self._init is not None:
            self._init = np.ascontiguousarray(self._init, dtype=np.int32)
            assert self._init.shape == (self.I, self.C)
        self._tun = None
        if tuning:
            self._tun = cwc_tuning(*[int(tuning.get(f, 0)) for f, _ in cwc_tuning._fields_])
        d = cwc_run_desc(
            run["seed"], self.I, self.R,
            None if self._rate is None else self._rate.ctypes.data,
            None if self._init is None else self._init.ctypes.data,
            run["dt"], self.K1, MODE_PERSISTENT if mode == "persistent" else MODE_PLAIN,
            int(want_traj), int(want_digest), run["count_cap"], run["max_events"],
            ctypes.pointer(self._tun) if self._tun is not None else None)
        self.want_traj = want_traj
        h = ctypes.c_void_p()
        check(L.cwc_run_submit(ctx.h, model.h, ctypes.byref(d),
                               _stream_handle(stream), ctypes.byref(h)))
        self.h = h

    def relaunch(self, stream=None):
        check(load().cwc_run_relaunch(self.h, _stream_handle(stream)))

    def done(self) -> bool:
        v = ctypes.c_int()
        check(load().cwc_run_query(self.h, ctypes.byref(v)))
        return bool(v.value)

    def wait(self):
        check(load().cwc_run_wait(self.h))
        return self

    def wait_for(self, timeout_s: float) -> bool:
        """cwc_run_wait_for: True once the launch has ended, False if it is
        still running after timeout_s seconds."""
        code = load().cwc_run_wait_for(self.h, float(timeout_s))
        if code == -5:
            return False
        check(code)
        return True

    def elapsed_ms(self):
        a, b = ctypes.c_float(), ctypes.c_float()
        check(load().cwc_run_elapsed(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def kernel_name(self) -> str:
        """Name of the simulation kernel this run dispatches."""
        L = load()
        n = ctypes.c_size_t()
        check(L.cwc_run_kernel_name(self.h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        check(L.cwc_run_kernel_name(self.h, buf, n.value, ctypes.byref(n)))
        return buf.value.decode()

    def stats(self):
        mean = np.empty((self.I, self.K1, self.C), np.float64)
        var = np.empty_like(mean)
        n = np.empty((self.I, self.K1), np.int64)
        check(load().cwc_run_fetch_stats(self.h, mean.ctypes.data, var.ctypes.data,
                                         n.ctypes.data, 0))
        return mean, var, n

    def moments(self):
        s1 = np.empty((self.I, self.K1, self.C), np.uint64)
        hi, lo = np.empty_like(s1), np.empty_like(s1)
        n = np.empty((self.I, self.K1), np.int64)
        check(load().cwc_run_fetch_moments(self.h, s1.ctypes.data, hi.ctypes.data,
                                           lo.ctypes.data, n.ctypes.data, 0))
        return s1, hi, lo, n

    def counters(self):
        G, C = self.G, self.C
        out = {"events": np.empty(G, np.int64), "status": np.empty(G, np.uint8),
               "digest": np.empty(G, np.uint64), "t_final": np.empty(G, np.float64),
               "n_recorded": np.empty(G, np.int32),
               "final_counts": np.empty((G, C), np.int32)}
        check(load().cwc_run_fetch_counters(
            self.h, *[out[k].ctypes.data for k in ("events", "status", "digest", "t_final",
                                                   "n_recorded", "final_counts")], 0))
        return out

    def trajectories(self, out=None):
        """Samples [K+1][C][G] int32 (trajectory fastest).  With ``out`` (a
        contiguous int32 device tensor of that shape) they are copied device
        to device into it and it is returned."""
        if out is not None:
            assert out.is_cuda and out.dtype.itemsize == 4 and out.is_contiguous()
            assert tuple(out.shape) == (self.K1, self.C, self.G)
            check(load().cwc_run_fetch_trajectories(self.h, out.data_ptr(), 1))
            return out
        t = np.empty((self.K1, self.C, self.G), np.int32)
        check(load().cwc_run_fetch_trajectories(self.h, t.ctypes.data, 0))
        return t

    def term(self):
        """General models: the final term [G][max_comp][alive, label, parent,
        wrap NS, content NS]."""
        m = self.model
        t = np.empty((self.G, m.max_comp, 3 + 2 * m.n_species), np.int32)
        check(load().cwc_run_fetch_term(self.h, t.ctypes.data, 0))
        return t

    def close(self):
        if getattr(self, "h", None):
            load().cwc_run_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_SCRATCH_BYTES = 32 << 20


def run_into(ctx: "Context", model: "Model", run: Dict, out: Dict, mode="plain",
             want_digest=False, tuning: Optional[Dict] = None, rate_table=None,
             init_table=None, stream=None):
    """cwc_run_into: the run on `stream` with no device allocation by the
    library.  ``out`` maps the output names of cwc_run_outputs (mean, var,
    n, events, status, digest, t_final, n_recorded, final_counts) to device
    tensors of the documented shapes and dtypes; ``rate_table`` /
    ``init_table`` are device tensors or None (the model's own).  Returns
    once the work is enqueued."""
    L = load()
    tun = None
    if tuning:
        tun = cwc_tuning(*[int(tuning.get(f, 0)) for f, _ in cwc_tuning._fields_])
    d = cwc_run_desc(
        run["seed"], run["n_instances"], run["replicas"],
        None if rate_table is None else rate_table.data_ptr(),
        None if init_table is None else init_table.data_ptr(),
        run["dt"], run["n_samples"], MODE_PERSISTENT if mode == "persistent" else MODE_PLAIN,
        0, int(want_digest), run["count_cap"], run["max_events"],
        ctypes.pointer(tun) if tun is not None else None)
    o = cwc_run_outputs(*[out[f].data_ptr() if out.get(f) is not None else None
                          for f, _ in cwc_run_outputs._fields_])
    check(L.cwc_run_into(ctx.h, model.h, ctypes.byref(d), ctypes.byref(o),
                         _stream_handle(stream)))


class Stream:
    """cwc_stream_*: a run executed in windows of ``window`` sample points
    with bounded device memory; iterate to get each window's statistics."""

    def __init__(self, ctx: Context, model: Model, run: Dict, window: int,
                 want_digest=False, lanes_per_replica: int = 0, stream=None):
        self.ctx, self.model = ctx, model
        self.I, self.R = run["n_instances"], run["replicas"]
        self.G = self.I * self.R
        self.K1 = run["n_samples"]
        self.C = model.info["n_cells"]
        d, self._rate, self._init = _run_desc(run, want_digest)
        self._tun = None
        if lanes_per_replica:
            self._tun = cwc_tuning(*[int(lanes_per_replica) if f == "lanes_per_replica" else 0
                                     for f, _ in cwc_tuning._fields_])
            d.tuning = ctypes.pointer(self._tun)
        h = ctypes.c_void_p()
        check(load().cwc_stream_open(ctx.h, model.h, ctypes.byref(d), int(window),
                                     _stream_handle(stream), ctypes.byref(h)))
        self.h = h
        self.window = self.info()["window"]

    def next(self):
        """(k0, mean [I][rows][C], var, n [I][rows]) of the next window, or
        None once every window has been returned."""
        W = self.window
        mean = np.empty((self.I, W, self.C), np.float64)
        var = np.empty_like(mean)
        n = np.empty((self.I, W), np.int64)
        k0, rows = ctypes.c_int32(), ctypes.c_int32()
        check(load().cwc_stream_next(self.h, ctypes.byref(k0), ctypes.byref(rows),
                                     mean.ctypes.data, var.ctypes.data, n.ctypes.data, 0))
        r = rows.value
        if r == 0:
            return None
        # the library packs [I][rows][C] (and [I][rows]) contiguously
        flat_m = mean.ravel()[: self.I * r * self.C].reshape(self.I, r, self.C)
        flat_v = var.ravel()[: self.I * r * self.C].reshape(self.I, r, self.C)
        flat_n = n.ravel()[: self.I * r].reshape(self.I, r)
        return k0.value, flat_m.copy(), flat_v.copy(), flat_n.copy()

    def __iter__(self):
        while True:
            w = self.next()
            if w is None:
                return
            yield w

    def term(self):
        """General models: the final term [G][max_comp][alive, label, parent,
        wrap NS, content NS], once every window has been returned."""
        m = self.model
        t = np.empty((self.G, m.max_comp, 3 + 2 * m.n_species), np.int32)
        check(load().cwc_stream_fetch_term(self.h, t.ctypes.data, 0))
        return t

    def info(self) -> Dict:
        i = cwc_stream_info_t()
        check(load().cwc_stream_info(self.h, ctypes.byref(i)))
        return {"device_bytes": int(i.device_bytes), "window": i.window,
                "n_windows": i.n_windows, "windows_done": i.windows_done,
                "last_window_ms": float(i.last_window_ms), "kernel": i.kernel.decode()}

    def counters(self):
        G, C = self.G, self.C
        out = {"events": np.empty(G, np.int64), "status": np.empty(G, np.uint8),
               "digest": np.empty(G, np.uint64), "t_final": np.empty(G, np.float64),
               "n_recorded": np.empty(G, np.int32),
               "final_counts": np.empty((G, C), np.int32)}
        check(load().cwc_stream_fetch_counters(
            self.h, *[out[k].ctypes.data for k in ("events", "status", "digest", "t_final",
                                                   "n_recorded", "final_counts")], 0))
        return out

    def close(self):
        if getattr(self, "h", None):
            load().cwc_stream_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _run_desc(run: Dict, want_digest=False):
    """cwc_run_desc for a workloads.make_run dictionary (tables kept alive by
    the returned tuple)."""
    rate = run.get("rate_table")
    init = run.get("init_table")
    if rate is not None:
        rate = np.ascontiguousarray(rate, dtype=np.float64)
    if init is not None:
        init = np.ascontiguousarray(init, dtype=np.int32)
    d = cwc_run_desc(run["seed"], run["n_instances"], run["replicas"],
                     None if rate is None else rate.ctypes.data,
                     None if init is None else init.ctypes.data,
                     run["dt"], run["n_samples"], MODE_PERSISTENT, 0, int(want_digest),
                     run["count_cap"], run["max_events"], None)
    return d, rate, init


class Server:
    """cwc_server_*: continuous batching of jobs within an HBM budget."""

    def __init__(self, ctx: Context, hbm_budget: int, max_active: int = 64,
                 slice_events: int = 4096):
        h = ctypes.c_void_p()
        check(load().cwc_server_create(ctx.h, int(hbm_budget), int(max_active),
                                       int(slice_events), ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self.shapes = {}
        self.models = {}

    def set_policy(self, slice_samples: int = 0, predicted: bool = False,
                   resident: bool = False):
        """cwc_server_set_policy: slices of `slice_samples` sample points (0:
        draw-bounded only) and the predictive dispatch order; or resident
        kernels draining per-model queues of (job, trajectory) items."""
        policy = 2 if resident else (1 if predicted else 0)
        check(load().cwc_server_set_policy(self.h, int(slice_samples), policy))

    def submit(self, model: Model, run: Dict, want_digest=False) -> int:
        d, _r, _i = _run_desc(run, want_digest)
        jid = ctypes.c_uint64()
        check(load().cwc_server_submit(self.h, model.h, ctypes.byref(d), ctypes.byref(jid)))
        self.shapes[jid.value] = (run["n_instances"], run["replicas"], run["n_samples"],
                                  model.info["n_cells"])
        self.models[jid.value] = model
        return jid.value

    def poll(self, max_n=4096):
        ids = (ctypes.c_uint64 * max_n)()
        n = ctypes.c_int32()
        check(load().cwc_server_poll(self.h, ids, max_n, ctypes.byref(n)))
        return list(ids[:n.value])

    def wait_idle(self, timeout_s=600.0):
        check(load().cwc_server_wait_idle(self.h, float(timeout_s)))

    def info(self, jid):
        i = cwc_job_info()
        check(load().cwc_server_job_info(self.h, jid, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in cwc_job_info._fields_}

    def stats(self, jid):
        I, R, K1, C = self.shapes[jid]
        mean = np.empty((I, K1, C), np.float64)
        var = np.empty_like(mean)
        n = np.empty((I, K1), np.int64)
        check(load().cwc_server_fetch_stats(self.h, jid, mean.ctypes.data, var.ctypes.data,
                                            n.ctypes.data, 0))
        return mean, var, n

    def counters(self, jid):
        I, R, K1, C = self.shapes[jid]
        G = I * R
        out = {"events": np.empty(G, np.int64), "status": np.empty(G, np.uint8),
               "digest": np.empty(G, np.uint64), "t_final": np.empty(G, np.float64),
               "n_recorded": np.empty(G, np.int32),
               "final_counts": np.empty((G, C), np.int32)}
        check(load().cwc_server_fetch_counters(
            self.h, jid, *[out[k].ctypes.data for k in ("events", "status", "digest",
                                                        "t_final", "n_recorded",
                                                        "final_counts")], 0))
        return out

    def term(self, jid):
        """General models: a completed job's final terms [G][max_comp][alive,
        label, parent, wrap NS, content NS]."""
        I, R, K1, C = self.shapes[jid]
        m = self.models[jid]
        # a fixed-tree job: the library refuses it before writing anything
        shape = (I * R, m.max_comp, 3 + 2 * m.n_species) if hasattr(m, "max_comp") else (1,)
        t = np.empty(shape, np.int32)
        check(load().cwc_server_fetch_term(self.h, jid, t.ctypes.data, 0))
        return t

    def release(self, jid):
        check(load().cwc_server_release(self.h, jid))
        self.shapes.pop(jid, None)
        self.models.pop(jid, None)

    def server_stats(self):
        st = cwc_server_stats()
        check(load().cwc_server_get_stats(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in cwc_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            load().cwc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
