"""Python binding of liblbp.so (include/lbp.h): argument marshalling only.

Every step of belief propagation runs in the library's HIP kernels; this
module converts numpy arrays / torch tensors to pointers and error codes to
exceptions.  torch supplies device memory and the HIP stream: a Context uses
``torch.cuda.current_stream()`` unless told otherwise, so library work is
ordered with torch work on that stream.

Importing this module loads the library and fails loudly if it is missing;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbp.so")

LBP_OK, LBP_E_INVALID, LBP_E_OOM, LBP_E_HIP, LBP_E_STATE, LBP_E_BUDGET, LBP_E_NONFINITE, \
    LBP_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
ERROR_NAMES = {0: "LBP_OK", -1: "LBP_E_INVALID", -2: "LBP_E_OOM", -3: "LBP_E_HIP", -4: "LBP_E_STATE",
               -5: "LBP_E_BUDGET", -6: "LBP_E_NONFINITE", -7: "LBP_E_UNSUPPORTED"}


class LBPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERROR_NAMES.get(code, str(code)), msg))
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError("liblbp.so is not built (%s); run python -m paper_2202_04110_amd.build" % LIB_PATH)

# torch first: liblbp.so then binds to the HIP runtime torch already loaded
# (same soname), so streams and device pointers are shared with torch and
# one runtime serves the process whatever the import order.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)
_P = C.c_void_p


class GraphDesc(C.Structure):
    _fields_ = [
        ("num_vars", C.c_int32), ("var_num_states", _P), ("evidence", _P),
        ("num_factors", C.c_int32), ("factor_kind", _P), ("factor_edge_off", _P), ("edge_var", _P),
        ("factor_cfg_table", _P), ("num_cfg_tables", C.c_int32), ("cfg_table_num_cfgs", _P),
        ("cfg_table_arity", _P), ("cfg_table_off", _P), ("cfg_table_states", _P),
        ("logpot_off", _P), ("log_potentials", _P),
    ]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("lbp_last_error", C.c_char_p, [])
_sig("lbp_validate", C.c_int, [C.POINTER(GraphDesc), _P])
_sig("lbp_check_layout", C.c_int, [C.POINTER(GraphDesc), _P])
_sig("lbp_ctx_create", C.c_int, [C.c_int, _P, C.POINTER(_P)])
_sig("lbp_ctx_set_stream", C.c_int, [_P, _P])
_sig("lbp_ctx_synchronize", C.c_int, [_P])
_sig("lbp_ctx_use_graphs", C.c_int, [_P, C.c_int])
_sig("lbp_ctx_destroy", None, [_P])
_sig("lbp_graph_upload", C.c_int, [_P, C.POINTER(GraphDesc), C.POINTER(_P)])
_sig("lbp_graph_free", None, [_P])
_sig("lbp_graph_sizes", C.c_int, [_P, _P])
_sig("lbp_set_evidence", C.c_int, [_P, _P, C.c_int])
_sig("lbp_set_log_potentials", C.c_int, [_P, _P, C.c_int])
_sig("lbp_reset_messages", C.c_int, [_P])
_sig("lbp_run_bp", C.c_int, [_P, C.c_int32, C.c_float, C.c_float])
_sig("lbp_get_beliefs", C.c_int, [_P, _P, C.c_int, C.c_int])
_sig("lbp_decode_map", C.c_int, [_P, _P, C.c_int])
_sig("lbp_graph_status", C.c_int, [_P])
_sig("lbp_get_messages", C.c_int, [_P, _P, C.c_int])
_sig("lbp_set_messages", C.c_int, [_P, _P, C.c_int])
_sig("lbp_run_bp_record", C.c_int, [_P, C.c_int32, C.c_float, C.c_float, C.c_int32])
_sig("lbp_run_bp_backward", C.c_int, [_P, _P, _P, _P])
_sig("lbp_batch_create", C.c_int, [_P, _P, C.c_int32, C.POINTER(_P)])
_sig("lbp_batch_run", C.c_int, [_P, C.c_int32, C.c_float, C.c_float])
_sig("lbp_batch_use_fused", C.c_int, [_P, C.c_int])
_sig("lbp_batch_autotune", C.c_int, [_P, C.c_float, C.c_float, C.c_int32, C.POINTER(C.c_int32)])
_sig("lbp_batch_free", None, [_P])
_sig("lbp_run_bp_until", C.c_int, [_P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_int32,
                                   C.POINTER(C.c_int32), C.POINTER(C.c_float)])
_sig("lbp_run_bp_until_noalloc", C.c_int, [_P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_int32,
                                           C.POINTER(C.c_int32), C.POINTER(C.c_float)])
_sig("lbp_bandwidth_probe", C.c_int, [_P, C.c_int32, _P, _P, C.c_int64, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_float)])
_sig("lbp_sampler_create", C.c_int, [_P, C.c_int32, C.POINTER(_P)])
_sig("lbp_sampler_run", C.c_int, [_P, C.c_int32, C.c_float, C.c_float, _P, _P, _P])
_sig("lbp_sampler_free", None, [_P])


class Completion(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("status", C.c_int32), ("iters_done", C.c_int32),
                ("num_vars", C.c_int64), ("num_var_states", C.c_int64), ("num_logpots", C.c_int64),
                ("beliefs", C.POINTER(C.c_float)), ("map", C.POINTER(C.c_int32)),
                ("grad_logpot", C.POINTER(C.c_float)),
                ("t_arrival", C.c_double), ("t_ready", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("residual", C.c_float), ("reserved", C.c_int32)]


_sig("lbp_server_create", C.c_int, [_P, C.c_int64, C.c_int32, C.c_int32, C.POINTER(_P)])
_sig("lbp_server_create_host_only", C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.POINTER(_P)])
_sig("lbp_server_clock", C.c_double, [_P])
_sig("lbp_server_submit", C.c_int, [_P, C.POINTER(GraphDesc), C.c_int32, C.c_float, C.c_float, _P, C.c_int32,
                                    C.c_double, C.c_uint64])
_sig("lbp_server_submit_until", C.c_int, [_P, C.POINTER(GraphDesc), C.c_int32, C.c_float, C.c_float, C.c_float,
                                          C.c_int32, C.c_double, C.c_uint64])
_sig("lbp_server_cancel", C.c_int, [_P, C.c_uint64])
_sig("lbp_server_poll", C.c_int, [_P, C.POINTER(Completion), C.c_int32, C.POINTER(C.c_int32)])
_sig("lbp_server_drain", C.c_int, [_P, C.c_double])
_sig("lbp_server_stats", C.c_int, [_P, _P])
_sig("lbp_server_destroy", None, [_P])
_sig("lbp_graph_num_launches", C.c_int, [_P, C.POINTER(C.c_int32)])
_sig("lbp_graph_get_launch", C.c_int, [_P, C.c_int32, _P])
_sig("lbp_graph_set_launch", C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32])
_sig("lbp_graph_set_fused_launch", C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32])
_sig("lbp_autotune", C.c_int, [_P, C.c_float, C.c_float, C.c_int32, _P])
_sig("lbp_graph_use_resident", C.c_int, [_P, C.c_int])
_sig("lbp_graph_resident_state", C.c_int, [_P, _P])
_sig("lbp_graph_use_fused", C.c_int, [_P, C.c_int])
_sig("lbp_graph_fused_state", C.c_int, [_P, _P])
_sig("lbp_time_phase", C.c_int, [_P, C.c_int32, C.c_int32, C.c_float, C.c_float, C.POINTER(C.c_float)])

EXPORTS = [n for n in dir(_lib) if n.startswith("lbp_")]


def last_error() -> str:
    return (_lib.lbp_last_error() or b"").decode()


def check(rc):
    if rc != LBP_OK:
        raise LBPError(rc, last_error())
    return rc


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(_P)
    return C.c_void_p(a.data_ptr())  # torch tensor


def make_desc(spec):
    """lbp_graph_desc over a GraphSpec's arrays; returns (desc, keep-alive list)."""
    keep = [
        np.ascontiguousarray(spec.var_num_states, np.int32),
        np.ascontiguousarray(spec.evidence, np.float32),
        np.ascontiguousarray(spec.factor_kind, np.int32),
        np.ascontiguousarray(spec.factor_edge_off, np.int64),
        np.ascontiguousarray(spec.edge_var, np.int32),
        np.ascontiguousarray(spec.factor_cfg_table, np.int32),
        np.ascontiguousarray(spec.cfg_table_num_cfgs, np.int32),
        np.ascontiguousarray(spec.cfg_table_arity, np.int32),
        np.ascontiguousarray(spec.cfg_table_off, np.int64),
        np.ascontiguousarray(spec.cfg_table_states, np.int32),
        np.ascontiguousarray(spec.logpot_off, np.int64),
        np.ascontiguousarray(spec.log_potentials, np.float32),
    ]
    d = GraphDesc()
    d.num_vars = keep[0].shape[0]
    d.var_num_states = _ptr(keep[0])
    d.evidence = _ptr(keep[1])
    d.num_factors = keep[2].shape[0]
    d.factor_kind = _ptr(keep[2])
    d.factor_edge_off = _ptr(keep[3])
    d.edge_var = _ptr(keep[4])
    d.factor_cfg_table = _ptr(keep[5])
    d.num_cfg_tables = keep[6].shape[0]
    d.cfg_table_num_cfgs = _ptr(keep[6])
    d.cfg_table_arity = _ptr(keep[7])
    d.cfg_table_off = _ptr(keep[8])
    d.cfg_table_states = _ptr(keep[9])
    d.logpot_off = _ptr(keep[10])
    d.log_potentials = _ptr(keep[11])
    return d, keep


def validate(spec) -> dict:
    """Host-only validation (no GPU needed). Returns the sizes."""
    d, keep = make_desc(spec)
    sizes = np.zeros(6, np.int64)
    check(_lib.lbp_validate(C.byref(d), _ptr(sizes)))
    return dict(zip(("V", "VS", "F", "E", "ES", "Tn"), (int(x) for x in sizes)))


def check_layout(spec) -> dict:
    """Host-only replay of every kernel's addresses against the layout."""
    d, keep = make_desc(spec)
    info = np.zeros(4, np.int64)
    check(_lib.lbp_check_layout(C.byref(d), _ptr(info)))
    return dict(zip(("M", "VB", "P", "tiles"), (int(x) for x in info)))


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class Context:
    """A device and a HIP stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        torch.cuda.set_device(device)
        h = _P()
        check(_lib.lbp_ctx_create(device, _stream_handle(stream), C.byref(h)))
        self.h = h
        self.device = device

    def set_stream(self, stream):
        check(_lib.lbp_ctx_set_stream(self.h, _stream_handle(stream)))

    def synchronize(self):
        check(_lib.lbp_ctx_synchronize(self.h))

    def use_graphs(self, enable: bool):
        check(_lib.lbp_ctx_use_graphs(self.h, int(bool(enable))))

    def bandwidth_probe(self, kind: int, src, dst, nbytes: int, blocks: int, reps: int = 10) -> float:
        """Milliseconds per launch of a plain streaming kernel (kind 0 read,
        1 copy, 2 write, 3 five reads per write) over device buffers."""
        ms = C.c_float()
        check(_lib.lbp_bandwidth_probe(self.h, int(kind), _ptr(src) if src is not None else None, _ptr(dst),
                                       int(nbytes), int(blocks), int(reps), C.byref(ms)))
        return float(ms.value)

    def close(self):
        if self.h:
            _lib.lbp_ctx_destroy(self.h)
            self.h = None


def _is_dev(x):
    return x is not None and not isinstance(x, np.ndarray)


class Graph:
    """A factor graph uploaded to the device; messages persist across runs."""

    def __init__(self, ctx: Context, spec):
        d, keep = make_desc(spec)
        h = _P()
        check(_lib.lbp_graph_upload(ctx.h, C.byref(d), C.byref(h)))
        self.h = h
        self.ctx = ctx
        s = np.zeros(8, np.int64)
        check(_lib.lbp_graph_sizes(h, _ptr(s)))
        (self.V, self.VS, self.F, self.E, self.ES, self.Tn, self.device_bytes,
         self.padded_edge_states) = (int(x) for x in s)
        st = np.zeros(2, np.int32)
        check(_lib.lbp_graph_fused_state(h, _ptr(st)))
        self.fused = bool(st[0])

    def free(self):
        if getattr(self, "h", None):
            _lib.lbp_graph_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def run_bp(self, iters: int, damping: float, temperature: float):
        check(_lib.lbp_run_bp(self.h, int(iters), float(damping), float(temperature)))

    def run_bp_until(self, max_iters: int, damping: float, temperature: float, tol: float,
                     check_every: int = 1):
        """Iterates until the last iteration's largest message change is
        below tol (checked every check_every iterations) or max_iters; returns
        (iterations run, last residual)."""
        done = C.c_int32()
        res = C.c_float()
        check(_lib.lbp_run_bp_until(self.h, int(max_iters), float(damping), float(temperature), float(tol),
                                    int(check_every), C.byref(done), C.byref(res)))
        return int(done.value), float(res.value)

    def run_bp_until_noalloc(self, max_iters: int, damping: float, temperature: float, tol: float,
                             check_every: int = 1):
        """run_bp_until whose workspace is the library's fixed device array
        (no device allocation; graphs beyond it raise LBP_E_UNSUPPORTED)."""
        done = C.c_int32()
        res = C.c_float()
        check(_lib.lbp_run_bp_until_noalloc(self.h, int(max_iters), float(damping), float(temperature),
                                            float(tol), int(check_every), C.byref(done), C.byref(res)))
        return int(done.value), float(res.value)

    def reset_messages(self):
        check(_lib.lbp_reset_messages(self.h))

    def get_beliefs(self, normalized: bool = True, out=None):
        """Host numpy array (synchronous) unless ``out`` is a device tensor."""
        if out is None:
            out = np.zeros(self.VS, np.float32)
        check(_lib.lbp_get_beliefs(self.h, _ptr(out), int(bool(normalized)), int(_is_dev(out))))
        return out

    def decode_map(self, out=None):
        if out is None:
            out = np.zeros(self.V, np.int32)
        check(_lib.lbp_decode_map(self.h, _ptr(out), int(_is_dev(out))))
        return out

    def status(self):
        check(_lib.lbp_graph_status(self.h))

    def get_messages(self, out=None):
        if out is None:
            out = np.zeros(self.ES, np.float32)
        check(_lib.lbp_get_messages(self.h, _ptr(out), int(_is_dev(out))))
        return out

    def set_messages(self, values):
        if not _is_dev(values):
            values = np.ascontiguousarray(values, np.float32)
        check(_lib.lbp_set_messages(self.h, _ptr(values), int(_is_dev(values))))

    def set_evidence(self, values):
        if not _is_dev(values):
            values = np.ascontiguousarray(values, np.float32)
        check(_lib.lbp_set_evidence(self.h, _ptr(values), int(_is_dev(values))))

    def set_log_potentials(self, values):
        if not _is_dev(values):
            values = np.ascontiguousarray(values, np.float32)
        check(_lib.lbp_set_log_potentials(self.h, _ptr(values), int(_is_dev(values))))

    def run_bp_record(self, iters: int, damping: float, temperature: float, ckpt_every: int = 10):
        """Like run_bp, keeping checkpoints for backward (T > 0, enumeration factors)."""
        check(_lib.lbp_run_bp_record(self.h, int(iters), float(damping), float(temperature), int(ckpt_every)))

    def backward(self, grad_q, grad_logpot, grad_evidence=None):
        """dL/dphi and dL/dtheta of L = sum(grad_q * q) for the recorded run
        (all device tensors, float32, flat orders)."""
        check(_lib.lbp_run_bp_backward(self.h, _ptr(grad_q), _ptr(grad_logpot),
                                       _ptr(grad_evidence) if grad_evidence is not None else None))

    def launches(self):
        """Launch groups: dicts with phase, kind, a, b, wpb, swizzle, items, fused_wpb,
        fused_variant (bit 0 swizzle, bit 1 tables loaded before the belief
        gathers)."""
        n = C.c_int32()
        check(_lib.lbp_graph_num_launches(self.h, C.byref(n)))
        out = []
        for i in range(n.value):
            v = np.zeros(9, np.int32)
            check(_lib.lbp_graph_get_launch(self.h, i, _ptr(v)))
            out.append(dict(zip(("phase", "kind", "a", "b", "wpb", "swizzle", "items", "fused_wpb",
                                 "fused_variant"), (int(x) for x in v))))
        return out

    def set_fused_launch(self, i: int, wpb: int, variant: int):
        check(_lib.lbp_graph_set_fused_launch(self.h, int(i), int(wpb), int(variant)))

    def use_fused(self, enable: bool):
        check(_lib.lbp_graph_use_fused(self.h, int(bool(enable))))

    @property
    def fused_in_use(self) -> bool:
        st = np.zeros(2, np.int32)
        check(_lib.lbp_graph_fused_state(self.h, _ptr(st)))
        return bool(st[1])

    def use_resident(self, enable: bool):
        """lbp_run_bp in one workgroup with messages in LDS (bitwise the
        same); off by default, chosen by autotune when faster."""
        check(_lib.lbp_graph_use_resident(self.h, int(bool(enable))))

    @property
    def resident_state(self):
        """(applies, in use) of the resident solver."""
        st = np.zeros(2, np.int32)
        check(_lib.lbp_graph_resident_state(self.h, _ptr(st)))
        return bool(st[0]), bool(st[1])

    def set_launch(self, i: int, wpb: int, swizzle: int):
        check(_lib.lbp_graph_set_launch(self.h, int(i), int(wpb), int(swizzle)))

    def autotune(self, damping: float, temperature: float, reps: int = 20):
        """Times every candidate launch shape; returns the chosen ms per group."""
        n = len(self.launches())
        ms = np.zeros(max(1, n), np.float32)
        check(_lib.lbp_autotune(self.h, float(damping), float(temperature), int(reps), _ptr(ms)))
        return ms[:n]

    def time_phase(self, phase: int, reps: int, damping: float, temperature: float) -> float:
        ms = C.c_float()
        check(_lib.lbp_time_phase(self.h, int(phase), int(reps), float(damping), float(temperature),
                                  C.byref(ms)))
        return float(ms.value)


class Batch:
    """Graphs advanced together in shared launches (same bits as alone)."""

    def __init__(self, ctx: Context, graphs):
        self.graphs = list(graphs)
        arr = (_P * max(1, len(self.graphs)))(*[g.h for g in self.graphs])
        h = _P()
        check(_lib.lbp_batch_create(ctx.h, arr, len(self.graphs), C.byref(h)))
        self.h = h

    def run_bp(self, iters: int, damping: float, temperature: float):
        check(_lib.lbp_batch_run(self.h, int(iters), float(damping), float(temperature)))

    def use_fused(self, enable: bool):
        """Fused iterations over every graph (all must be fusable)."""
        check(_lib.lbp_batch_use_fused(self.h, int(bool(enable))))

    def autotune(self, damping: float, temperature: float, reps: int = 20) -> bool:
        """Tunes the batch's launch shapes (and fused vs two-phase iterations
        when every graph has them); returns whether fused iterations won."""
        fused = C.c_int32(0)
        check(_lib.lbp_batch_autotune(self.h, float(damping), float(temperature), int(reps), C.byref(fused)))
        return bool(fused.value)

    def free(self):
        if getattr(self, "h", None):
            _lib.lbp_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Sampler:
    """num_samples solves of one graph under perturbed evidence in shared
    launches (perturb-and-MAP: Gumbel noise, temperature 0).  The graph must
    outlive the sampler."""

    def __init__(self, graph: Graph, num_samples: int):
        self.graph = graph
        self.S = int(num_samples)
        h = _P()
        check(_lib.lbp_sampler_create(graph.h, self.S, C.byref(h)))
        self.h = h

    def run(self, iters: int, damping: float, temperature: float, noise, map_out=None, q_out=None):
        """noise: CUDA float32 tensor (num_samples, VS).  Returns the MAP
        states, a CUDA int32 tensor (num_samples, V) (and q_out, if given, holds
        (num_samples, VS) normalised beliefs).  Asynchronous on the context's
        stream."""
        import torch
        assert noise.is_cuda and noise.dtype == torch.float32 and noise.is_contiguous()
        assert noise.numel() == self.S * self.graph.VS
        if map_out is None:
            map_out = torch.empty((self.S, self.graph.V), device=noise.device, dtype=torch.int32)
        check(_lib.lbp_sampler_run(self.h, int(iters), float(damping), float(temperature), _ptr(noise),
                                   _ptr(map_out), _ptr(q_out) if q_out is not None else None))
        return map_out

    def free(self):
        if getattr(self, "h", None):
            _lib.lbp_sampler_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


SERVER_STATS = ("accepted", "finished", "completed", "rejected", "failed", "cancelled", "rounds",
                "resident", "queued", "max_resident", "arena_peak_bytes", "busy_us", "round_us", "prep_us",
                "prep_threads", "admit_us", "launch_us", "finish_us")


class Server:
    """Continuous-batching server (see lbp_server_* in include/lbp.h)."""

    def __init__(self, ctx=None, budget_bytes: int = 1 << 30, max_slots: int = 64, steps_per_round: int = 5,
                 host_only: bool = False):
        h = _P()
        if host_only:
            check(_lib.lbp_server_create_host_only(int(budget_bytes), int(max_slots), int(steps_per_round),
                                                   C.byref(h)))
        else:
            check(_lib.lbp_server_create(ctx.h, int(budget_bytes), int(max_slots), int(steps_per_round),
                                         C.byref(h)))
        self.h = h

    def clock(self) -> float:
        return float(_lib.lbp_server_clock(self.h))

    def submit(self, spec, iters: int, damping: float, temperature: float, grad_q=None, ckpt_every: int = 10,
               t_arrival: float = -1.0, req_id: int = 0, tol=None, check_every: int = 10):
        """tol (not None): the request stops once the residual measured every
        check_every of its iterations is below tol (lbp_server_submit_until;
        forward only), with at most `iters` iterations."""
        d, keep = make_desc(spec)
        if tol is not None:
            if grad_q is not None:
                raise ValueError("a request with tol cannot carry a gradient")
            check(_lib.lbp_server_submit_until(self.h, C.byref(d), int(iters), float(damping), float(temperature),
                                               float(tol), int(check_every), float(t_arrival), int(req_id)))
            return
        gq = None if grad_q is None else np.ascontiguousarray(grad_q, np.float32)
        check(_lib.lbp_server_submit(self.h, C.byref(d), int(iters), float(damping), float(temperature),
                                     _ptr(gq), int(ckpt_every), float(t_arrival), int(req_id)))

    def cancel(self, req_id: int):
        check(_lib.lbp_server_cancel(self.h, int(req_id)))

    def poll(self, max_n: int = 256):
        """Finished requests as dicts; outputs are copied into numpy arrays."""
        buf = (Completion * max_n)()
        n = C.c_int32()
        check(_lib.lbp_server_poll(self.h, buf, max_n, C.byref(n)))
        out = []
        for i in range(n.value):
            c = buf[i]
            rec = {"req_id": int(c.req_id), "status": int(c.status), "iters": int(c.iters_done),
                   "residual": float(c.residual), "t_arrival": c.t_arrival, "t_ready": c.t_ready,
                   "t_admit": c.t_admit, "t_done": c.t_done, "beliefs": None, "map": None, "grad_logpot": None}
            if c.beliefs:
                rec["beliefs"] = np.ctypeslib.as_array(c.beliefs, (c.num_var_states,)).copy()
                rec["map"] = np.ctypeslib.as_array(c.map, (c.num_vars,)).copy()
            if c.grad_logpot:
                rec["grad_logpot"] = np.ctypeslib.as_array(c.grad_logpot, (c.num_logpots,)).copy()
            out.append(rec)
        return out

    def drain(self, timeout: float = 600.0):
        check(_lib.lbp_server_drain(self.h, float(timeout)))

    def stats(self) -> dict:
        s = np.zeros(len(SERVER_STATS), np.int64)
        check(_lib.lbp_server_stats(self.h, _ptr(s)))
        return dict(zip(SERVER_STATS, (int(x) for x in s)))

    def close(self):
        if getattr(self, "h", None):
            _lib.lbp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
