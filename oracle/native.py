"""ctypes wrapper of the C oracle ``fsg_oracle.c`` (test infrastructure only).

The wrapper only marshals arguments; all arithmetic is in the C file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsg_oracle.c")
_LIB = os.path.join(_HERE, "libfsg_oracle.so")

IC, SI, SIS, SIR, LT, SEIR, SEIS, SWIR = 0, 1, 2, 3, 4, 5, 6, 7
IC_UNIFORM, IC_WEIGHTED_CASCADE, IC_PER_EDGE = 0, 1, 2
DOM_IC_EDGE, DOM_NODE_STEP, DOM_LT_THRESH = 1, 2, 3
MODEL_NAMES = {"ic": IC, "si": SI, "sis": SIS, "sir": SIR, "lt": LT, "seir": SEIR, "seis": SEIS,
               "swir": SWIR}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, FP contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.orc_philox4x32_10.restype = None
        lib.orc_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_uint32]
        lib.orc_draw.restype = ctypes.c_uint32
        lib.orc_draw_many.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p]
        lib.orc_draw_many.restype = None
        lib.orc_thr.argtypes = [ctypes.c_double]
        lib.orc_thr.restype = ctypes.c_uint32
        lib.orc_sir_table.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_void_p]
        lib.orc_sir_table.restype = None
        lib.orc_simulate.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_double,
            ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_uint64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
            ctypes.POINTER(ctypes.c_int32), ctypes.c_int]
        lib.orc_simulate.restype = ctypes.c_int
        lib.orc_ic_live_edge.argtypes = [
            ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), ctypes.c_int]
        lib.orc_ic_live_edge.restype = ctypes.c_int
        lib.orc_hk.argtypes = [ctypes.c_float, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                               ctypes.c_int]
        lib.orc_hk.restype = ctypes.c_int
        lib.orc_whk.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                ctypes.c_int]
        lib.orc_whk.restype = ctypes.c_int
        lib.orc_hk_rows.argtypes = [ctypes.c_float, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.orc_hk_rows.restype = ctypes.c_int
        lib.orc_set_verbose.argtypes = [ctypes.c_int]
        lib.orc_set_verbose.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key):
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib.orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def draw(rng_key, dom, unit, g, step):
    return int(_load().orc_draw(rng_key, dom, unit, g, step))


def draw_many(rng_key, dom, unit, g, step):
    unit = np.ascontiguousarray(unit, dtype=np.uint64)
    g = np.ascontiguousarray(np.broadcast_to(g, unit.shape), dtype=np.uint64)
    step = np.ascontiguousarray(np.broadcast_to(step, unit.shape), dtype=np.uint32)
    out = np.empty(unit.shape, dtype=np.uint32)
    _load().orc_draw_many(rng_key, dom, _ptr(unit), _ptr(g), _ptr(step), unit.size, _ptr(out))
    return out


def thr(p):
    return int(_load().orc_thr(float(p)))


def sir_table(beta, length):
    out = np.empty(int(length), dtype=np.uint32)
    _load().orc_sir_table(float(beta), int(length), _ptr(out))
    return out


def _csr(ptr, src):
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    src = np.ascontiguousarray(src, dtype=np.int32)
    return ptr, src


def simulate(model, ptr, src, seeds, B, rng_key, *, p=0.0, ic_prob=IC_UNIFORM, edge_p=None,
             beta=0.0, gamma=0.0, alpha=0.0, max_steps=-1, replicate_offset=0,
             want_states=True, nthreads=0):
    """Plain batched simulation.  Returns (states [n,B] uint8 or None, counts [n] uint32,
    steps_run, absorbed)."""
    lib = _load()
    if isinstance(model, str):
        model = MODEL_NAMES[model]
    ptr, src = _csr(ptr, src)
    n = ptr.size - 1
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    ep = None if edge_p is None else np.ascontiguousarray(edge_p, dtype=np.float64)
    states = np.empty((n, B), dtype=np.uint8) if want_states else None
    counts = np.empty(n, dtype=np.uint32)
    steps = ctypes.c_int64(0)
    absorbed = ctypes.c_int32(0)
    rc = lib.orc_simulate(model, ic_prob, float(p), _ptr(ep), float(beta), float(gamma),
                          float(alpha), int(max_steps), n, _ptr(ptr), _ptr(src), _ptr(seeds), seeds.size,
                          int(B), int(replicate_offset), int(rng_key) & (2**64 - 1),
                          _ptr(states), _ptr(counts), ctypes.byref(steps),
                          ctypes.byref(absorbed), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return states, counts, int(steps.value), int(absorbed.value)


def ic_live_edge(ptr, src, seeds, B, rng_key, *, p=0.0, ic_prob=IC_UNIFORM, edge_p=None,
                 max_steps=-1, replicate_offset=0, want_states=True, want_dist=False,
                 nthreads=0, verbose=False):
    """IC via BFS in the live-edge graph.  Returns (states, counts, dist, steps_run, absorbed)."""
    lib = _load()
    lib.orc_set_verbose(1 if verbose else 0)
    ptr, src = _csr(ptr, src)
    n = ptr.size - 1
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    ep = None if edge_p is None else np.ascontiguousarray(edge_p, dtype=np.float64)
    states = np.empty((n, B), dtype=np.uint8) if want_states else None
    dist = np.empty((n, B), dtype=np.int32) if want_dist else None
    counts = np.empty(n, dtype=np.uint32)
    steps = ctypes.c_int64(0)
    absorbed = ctypes.c_int32(0)
    rc = lib.orc_ic_live_edge(ic_prob, float(p), _ptr(ep), int(max_steps), n, _ptr(ptr),
                              _ptr(src), _ptr(seeds), seeds.size, int(B), int(replicate_offset),
                              int(rng_key) & (2**64 - 1), _ptr(states), _ptr(counts), _ptr(dist),
                              ctypes.byref(steps), ctypes.byref(absorbed), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return states, counts, dist, int(steps.value), int(absorbed.value)


def hk(ptr, src, h0, eps, max_steps, nthreads=0):
    """Hegselmann-Krause from opinions h0 [n, B] (float32).  Returns (h [n, B]
    float32, steps_run, converged)."""
    lib = _load()
    ptr, src = _csr(ptr, src)
    n = ptr.size - 1
    h = np.ascontiguousarray(h0, dtype=np.float32).copy()
    assert h.shape[0] == n
    B = h.shape[1]
    steps = ctypes.c_int64(0)
    conv = ctypes.c_int32(0)
    rc = lib.orc_hk(float(np.float32(eps)), int(max_steps), n, _ptr(ptr), _ptr(src), B, _ptr(h),
                    ctypes.byref(steps), ctypes.byref(conv), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return h, int(steps.value), int(conv.value)


def whk(ptr, src, h0, eps, mu, max_steps, nthreads=0):
    """Weighted Hegselmann-Krause: each node moves the fraction mu of the way
    to its HK mean, (1 - mu) h + mu m in float32.  Returns (h, steps_run,
    converged) as :func:`hk`."""
    lib = _load()
    ptr, src = _csr(ptr, src)
    n = ptr.size - 1
    h = np.ascontiguousarray(h0, dtype=np.float32).copy()
    assert h.shape[0] == n
    B = h.shape[1]
    steps = ctypes.c_int64(0)
    conv = ctypes.c_int32(0)
    rc = lib.orc_whk(float(np.float32(eps)), float(np.float32(mu)), int(max_steps), n, _ptr(ptr),
                     _ptr(src), B, _ptr(h), ctypes.byref(steps), ctypes.byref(conv), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return h, int(steps.value), int(conv.value)


def hk_rows(ptr, src, h, eps, rows):
    """One Hegselmann-Krause step of the listed rows from opinions h [n, B];
    returns float32 [len(rows), B]."""
    lib = _load()
    ptr, src = _csr(ptr, src)
    n = ptr.size - 1
    h = np.ascontiguousarray(h, dtype=np.float32)
    assert h.shape[0] == n
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.size, h.shape[1]), dtype=np.float32)
    rc = lib.orc_hk_rows(float(np.float32(eps)), n, _ptr(ptr), _ptr(src), h.shape[1], _ptr(h),
                         _ptr(rows), rows.size, _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out
