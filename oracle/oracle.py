"""ctypes front of the FP64 C oracle (``lbp_oracle.c``) -- test infrastructure only.

Takes any object with the flat-array fields of a factor graph (see
``lbp_oracle.c`` for the method) and hands them to the C code; FP32 values are
widened to FP64 there, so only arithmetic precision differs from the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbp_oracle.c")
_LIB = os.path.join(_HERE, "liblbp_oracle.so")
_lib = None
_libs = {}


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP on)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def oracle_available() -> bool:
    try:
        _load()
        return True
    except Exception:
        return False


def _load(path=None):
    """Loads the oracle library (by default the one built from lbp_oracle.c;
    ``path`` selects another build of the same source, e.g. a mutated copy in
    the mutation test)."""
    global _lib
    if path is None:
        if _lib is not None:
            return _lib
        build_oracle()
        path = _LIB
    if path in _libs:
        return _libs[path]
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.og_create.restype = P
    lib.og_create.argtypes = [C.c_int32, P, P, C.c_int32, P, P, P, P, C.c_int32, P, P, P, P, P]
    lib.og_free.argtypes = [P]
    lib.og_run.restype = C.c_int
    lib.og_run.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_int32, P, P]
    lib.og_update.restype = C.c_int
    lib.og_update.argtypes = [P, C.c_double, P, P]
    lib.og_beliefs.restype = C.c_int
    lib.og_beliefs.argtypes = [P, P, C.c_double, P, P, P]
    lib.og_score.restype = C.c_double
    lib.og_score.argtypes = [P, P]
    lib.og_backward.restype = C.c_int
    lib.og_backward.argtypes = [P, C.c_int32, C.c_double, C.c_double, P, P, P, P, P]
    lib.og_num_edge_states.restype = C.c_int64
    lib.og_num_edge_states.argtypes = [P]
    lib.og_num_var_states.restype = C.c_int64
    lib.og_num_var_states.argtypes = [P]
    _libs[path] = lib
    if path == _LIB:
        _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class OracleGraph:
    """A factor graph loaded into the oracle."""

    def __init__(self, g, lib_path=None):
        lib = self._lib = _load(lib_path)
        self._keep = [
            np.ascontiguousarray(g.var_num_states, np.int32),
            np.ascontiguousarray(g.evidence, np.float32),
            np.ascontiguousarray(g.factor_kind, np.int32),
            np.ascontiguousarray(g.factor_edge_off, np.int64),
            np.ascontiguousarray(g.edge_var, np.int32),
            np.ascontiguousarray(g.factor_cfg_table, np.int32),
            np.ascontiguousarray(g.cfg_table_num_cfgs, np.int32),
            np.ascontiguousarray(g.cfg_table_off, np.int64),
            np.ascontiguousarray(g.cfg_table_states, np.int32),
            np.ascontiguousarray(g.logpot_off, np.int64),
            np.ascontiguousarray(g.log_potentials, np.float32),
        ]
        k = self._keep
        self.V = int(k[0].shape[0])
        self.F = int(k[2].shape[0])
        self.Tn = int(k[10].shape[0])
        self.h = lib.og_create(self.V, _p(k[0]), _p(k[1]), self.F, _p(k[2]), _p(k[3]),
                               _p(k[4]), _p(k[5]), int(k[6].shape[0]), _p(k[6]), _p(k[7]),
                               _p(k[8]), _p(k[9]), _p(k[10]))
        if not self.h:
            raise MemoryError("oracle graph allocation failed")
        self.ES = int(lib.og_num_edge_states(self.h))
        self.VS = int(lib.og_num_var_states(self.h))
        self.last_seconds = 0.0

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.og_free(self.h)
            self.h = None

    def zero_messages(self) -> np.ndarray:
        return np.zeros(self.ES, np.float64)

    def run(self, iters: int, damping: float, temperature: float, m0=None, threads: int = 1,
            residuals: bool = False):
        """Runs ``iters`` iterations from m0 (default zeros). Returns the
        messages (and the per-iteration max-abs change when ``residuals``)."""
        m = self.zero_messages() if m0 is None else np.array(m0, np.float64, copy=True)
        assert m.shape == (self.ES,)
        res = np.zeros(max(iters, 1), np.float64)
        t0 = time.perf_counter()
        rc = self._lib.og_run(self.h, int(iters), float(damping), float(temperature), int(threads),
                         _p(m), _p(res) if residuals else None)
        self.last_seconds = time.perf_counter() - t0
        if rc != 0:
            raise RuntimeError("oracle run failed (%d)" % rc)
        return (m, res[:iters]) if residuals else m

    def update(self, m, temperature: float) -> np.ndarray:
        """Undamped, unnormalised factor-to-variable update u(m)."""
        m = np.ascontiguousarray(m, np.float64)
        u = np.zeros(self.ES, np.float64)
        if self._lib.og_update(self.h, float(temperature), _p(m), _p(u)) != 0:
            raise RuntimeError("oracle update failed")
        return u

    def beliefs(self, m, temperature: float):
        """Returns (B, q, map) from messages m."""
        m = np.ascontiguousarray(m, np.float64)
        B = np.zeros(self.VS, np.float64)
        q = np.zeros(self.VS, np.float64)
        mp = np.zeros(self.V, np.int32)
        if self._lib.og_beliefs(self.h, _p(m), float(temperature), _p(B), _p(q), _p(mp)) != 0:
            raise RuntimeError("oracle beliefs failed")
        return B, q, mp

    def score(self, x) -> float:
        x = np.ascontiguousarray(x, np.int32)
        assert x.shape == (self.V,)
        return float(self._lib.og_score(self.h, _p(x)))

    def backward(self, iters: int, damping: float, temperature: float, grad_q, m0=None):
        """Gradient of sum(grad_q * q) w.r.t. (log_potentials, evidence, m0)."""
        m0 = self.zero_messages() if m0 is None else np.ascontiguousarray(m0, np.float64)
        gq = np.ascontiguousarray(grad_q, np.float64)
        gphi = np.zeros(self.Tn, np.float64)
        gth = np.zeros(self.VS, np.float64)
        gm0 = np.zeros(self.ES, np.float64)
        rc = self._lib.og_backward(self.h, int(iters), float(damping), float(temperature), _p(m0),
                              _p(gq), _p(gphi), _p(gth), _p(gm0))
        if rc != 0:
            raise RuntimeError("oracle backward failed (%d)" % rc)
        return gphi, gth, gm0

    def solve(self, iters, damping, temperature, threads=1):
        """Messages, normalised beliefs q, MAP and residual history."""
        m, res = self.run(iters, damping, temperature, threads=threads, residuals=True)
        _, q, mp = self.beliefs(m, temperature)
        return {"m": m, "q": q, "map": mp, "resid": res}
