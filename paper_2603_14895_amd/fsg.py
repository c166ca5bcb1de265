"""Python binding of libfsg (declarations in include/fsg.h).

Argument marshalling only: every step of the propagation runs in the HIP
library.  PyTorch supplies device memory (workspaces and outputs) and the
stream.  If the shared library is missing this module raises on import of the
library -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsg.so")

FSG_OK, FSG_EINVAL, FSG_ENOMEM, FSG_EDEVICE, FSG_EUNSUPPORTED, FSG_EWORKSPACE = 0, -1, -2, -3, -4, -5
FSG_IC, FSG_SI, FSG_SIS, FSG_SIR, FSG_LT, FSG_SEIR, FSG_SEIS, FSG_SWIR = 0, 1, 2, 3, 4, 5, 6, 7
FSG_IC_UNIFORM, FSG_IC_WEIGHTED_CASCADE, FSG_IC_PER_EDGE = 0, 1, 2
MODELS = {"ic": FSG_IC, "si": FSG_SI, "sis": FSG_SIS, "sir": FSG_SIR, "lt": FSG_LT,
          "seir": FSG_SEIR, "seis": FSG_SEIS, "swir": FSG_SWIR}
IC_PROBS = {"uniform": FSG_IC_UNIFORM, "weighted_cascade": FSG_IC_WEIGHTED_CASCADE,
            "per_edge": FSG_IC_PER_EDGE}


class FsgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfsg error {code}: {msg}")
        self.code = code


class fsg_params(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("ic_prob", ctypes.c_int32), ("p", ctypes.c_double),
                ("edge_p", ctypes.c_void_p), ("beta", ctypes.c_double),
                ("gamma", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("alpha", ctypes.c_double)]


class fsg_run_info(ctypes.Structure):
    _fields_ = [("steps_run", ctypes.c_int64), ("absorbed", ctypes.c_int32),
                ("tail_steps", ctypes.c_int32), ("step_kernel_ms", ctypes.c_double),
                ("step_launches", ctypes.c_int64), ("setup_ms", ctypes.c_double),
                ("finalize_ms", ctypes.c_double), ("philox_calls", ctypes.c_int64)]


class fsg_schedule(ctypes.Structure):
    _fields_ = [("row_lanes", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("tile_edges", ctypes.c_int32), ("heavy_threshold", ctypes.c_int32),
                ("steps_per_sync", ctypes.c_int32), ("time_kernels", ctypes.c_int32),
                ("kernel_variant", ctypes.c_int32), ("options", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


OPT_WIDE_OFFSETS = 1  # FSG_OPT_WIDE_OFFSETS
OPT_COUNT_DRAWS = 2   # FSG_OPT_COUNT_DRAWS
OPT_REUSE_WORKSPACE = 4  # FSG_OPT_REUSE_WORKSPACE
OPT_TAIL_OFF = 8  # FSG_OPT_TAIL_OFF
OPT_TAIL_ALWAYS = 16  # FSG_OPT_TAIL_ALWAYS


CALIB_TERMS = 9


class fsg_spread_gate(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("min_seeds", ctypes.c_int64),
                ("calibrated", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("calib", ctypes.c_double * CALIB_TERMS)]


def make_gate(tau: float = float("inf"), min_seeds: int = 0, calib=None) -> fsg_spread_gate:
    g = fsg_spread_gate()
    g.tau = float(tau)
    g.min_seeds = int(min_seeds)
    g.calibrated = 0 if calib is None else 1
    if calib is not None:
        c = [float(x) for x in calib]
        if len(c) != CALIB_TERMS:
            raise ValueError(f"calibration needs {CALIB_TERMS} coefficients")
        for i, x in enumerate(c):
            g.calib[i] = x
    return g


class fsg_job(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("prm", fsg_params), ("seeds", ctypes.c_void_p),
                ("n_seeds", ctypes.c_int64), ("B", ctypes.c_int64),
                ("replicate_offset", ctypes.c_int64), ("rng_key", ctypes.c_uint64),
                ("sched", fsg_schedule), ("final_states", ctypes.c_void_p),
                ("infected_counts", ctypes.c_void_p)]


_lib = None
_VP, _I64, _I32, _U32, _U64, _SZ = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t)

# name -> (restype, argtypes)
_SIGS = {
    "fsg_abi_version": (ctypes.c_int, []),
    "fsg_last_error": (ctypes.c_char_p, []),
    "fsg_graph_create": (ctypes.c_int, [_I64, _I64, _VP, _VP, ctypes.POINTER(_VP)]),
    "fsg_graph_workspace_size": (ctypes.c_int, [_VP, ctypes.POINTER(_SZ)]),
    "fsg_graph_bind": (ctypes.c_int, [_VP, _VP, _SZ, _VP]),
    "fsg_graph_out_workspace_size": (ctypes.c_int, [_VP, ctypes.POINTER(_SZ)]),
    "fsg_graph_bind_out": (ctypes.c_int, [_VP, _VP, _SZ, _VP]),
    "fsg_graph_stats": (ctypes.c_int, [_VP, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                       ctypes.POINTER(_I64)]),
    "fsg_graph_destroy": (ctypes.c_int, [_VP]),
    "fsg_default_schedule": (ctypes.c_int, [_VP, ctypes.POINTER(fsg_params), _I64,
                                            ctypes.POINTER(fsg_schedule)]),
    "fsg_sim_workspace_size": (ctypes.c_int, [_VP, ctypes.POINTER(fsg_params), _I64,
                                              ctypes.POINTER(fsg_schedule), ctypes.POINTER(_SZ)]),
    "fsg_simulate": (ctypes.c_int, [_VP, ctypes.POINTER(fsg_params), _VP, _I64, _I64, _I64, _U64,
                                    ctypes.POINTER(fsg_schedule), _VP, _SZ, _VP, _VP,
                                    ctypes.POINTER(fsg_run_info), _VP]),
    "fsg_simulate_noalloc_limit": (_SZ, []),
    "fsg_simulate_noalloc": (ctypes.c_int, [_VP, ctypes.POINTER(fsg_params), _VP, _I64, _I64,
                                            _I64, _U64, ctypes.POINTER(fsg_schedule), _VP, _VP,
                                            ctypes.POINTER(fsg_run_info), _VP]),
    "fsg_session_begin": (ctypes.c_int, [_VP, ctypes.POINTER(fsg_params), _VP, _I64, _I64, _I64,
                                         _U64, ctypes.POINTER(fsg_schedule), _VP, _SZ, _VP,
                                         ctypes.POINTER(_VP)]),
    "fsg_session_step": (ctypes.c_int, [_VP, _I64, _VP, ctypes.POINTER(fsg_run_info), _VP]),
    "fsg_session_read": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "fsg_session_end": (ctypes.c_int, [_VP]),
    "fsg_philox4x32_10": (ctypes.c_int, [_VP, _U32, _U32, _VP, _I64, _VP]),
    "fsg_plan_row_tiles": (ctypes.c_int, [_VP, _I64, _I64, _I64, _I64, _VP, ctypes.POINTER(_I64)]),
    "fsg_batch_plan": (ctypes.c_int, [ctypes.POINTER(fsg_job), _I32, _I32, ctypes.POINTER(_VP),
                                      ctypes.POINTER(_SZ)]),
    "fsg_batch_run": (ctypes.c_int, [_VP, _VP, _SZ, ctypes.POINTER(fsg_run_info),
                                     ctypes.POINTER(ctypes.c_double), _VP]),
    "fsg_plan_destroy": (ctypes.c_int, [_VP]),
    "fsg_batch_set_launch": (ctypes.c_int, [_VP, _I32]),
    "fsg_batch_autotune_workspace_size": (ctypes.c_int, [ctypes.POINTER(fsg_job), _I32,
                                                         ctypes.POINTER(_SZ)]),
    "fsg_batch_autotune": (ctypes.c_int, [ctypes.POINTER(fsg_job), _I32, _I32, _VP, _SZ,
                                          ctypes.POINTER(fsg_job), ctypes.POINTER(_I32),
                                          ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I32),
                                          _VP]),
    "fsg_gnn_create": (ctypes.c_int, [_I32, _I32, _U64, ctypes.POINTER(_VP)]),
    "fsg_gnn_destroy": (ctypes.c_int, [_VP]),
    "fsg_gnn_param_count": (ctypes.c_int, [_VP, ctypes.POINTER(_I64)]),
    "fsg_gnn_state_size": (ctypes.c_int, [_VP, ctypes.POINTER(_SZ)]),
    "fsg_gnn_bind": (ctypes.c_int, [_VP, _VP, _SZ, _VP]),
    "fsg_gnn_workspace_size": (ctypes.c_int, [_VP, _VP, _I32, ctypes.POINTER(_SZ)]),
    "fsg_gnn_forward": (ctypes.c_int, [_VP, _VP, _I32, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "fsg_gnn_train_step": (ctypes.c_int, [_VP, _VP, _VP, _I32, _VP, _VP, _VP, ctypes.c_float, _I32,
                                          ctypes.POINTER(ctypes.c_float), _VP, _SZ, _VP]),
    "fsg_gnn_get_params": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "fsg_gnn_set_params": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "fsg_gnn_get_grads": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "fsg_gnn_apply_update": (ctypes.c_int, [_VP, _VP, ctypes.c_float, _VP]),
    "fsg_gnn_get_state": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(_I64), _I64, _VP]),
    "fsg_estimate_spread": (ctypes.c_int, [_VP, _I32, _VP, _VP, _I64, ctypes.c_double,
                                           ctypes.c_double, _I64, ctypes.POINTER(fsg_spread_gate),
                                           _I64, _U64, _VP, _SZ, _VP, _SZ, _VP,
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int32), _VP]),
    "fsg_hk_workspace_size": (ctypes.c_int, [_VP, _I64, ctypes.POINTER(fsg_schedule),
                                             ctypes.POINTER(_SZ)]),
    "fsg_hk": (ctypes.c_int, [_VP, ctypes.c_float, _I64, _I64, _VP, ctypes.POINTER(fsg_schedule),
                              _VP, _SZ, ctypes.c_float, _VP, ctypes.POINTER(fsg_run_info), _VP]),
    "fsg_whk": (ctypes.c_int, [_VP, ctypes.c_float, ctypes.c_float, _I64, _I64, _VP,
                               ctypes.POINTER(fsg_schedule), _VP, _SZ, ctypes.c_float, _VP,
                               ctypes.POINTER(fsg_run_info), _VP]),
    "fsg_autotune_workspace_size": (ctypes.c_int, [_VP, ctypes.POINTER(fsg_params), _I64, _I32,
                                                   ctypes.POINTER(_SZ)]),
    "fsg_autotune": (ctypes.c_int, [_VP, ctypes.POINTER(fsg_params), _VP, _I64, _I64, _U64, _I32,
                                    _I32, ctypes.c_char_p, _VP, _SZ, ctypes.POINTER(fsg_schedule),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), _VP]),
}


def exported_names():
    return list(_SIGS)


def lib():
    """Load libfsg.so (built in-tree by paper_2603_14895_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2603_14895_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != FSG_OK:
        raise FsgError(rc, lib().fsg_last_error().decode())


# ---------------------------------------------------------------- raw calls --

def fsg_abi_version() -> int:
    return lib().fsg_abi_version()


def fsg_last_error() -> str:
    return lib().fsg_last_error().decode()


def fsg_graph_create(n, nnz, in_ptr_addr, in_src_addr) -> int:
    h = ctypes.c_void_p()
    _check(lib().fsg_graph_create(n, nnz, in_ptr_addr, in_src_addr, ctypes.byref(h)))
    return h.value


def fsg_graph_workspace_size(g) -> int:
    b = ctypes.c_size_t()
    _check(lib().fsg_graph_workspace_size(g, ctypes.byref(b)))
    return b.value


def fsg_graph_bind(g, dev_ws, ws_bytes, stream=None):
    _check(lib().fsg_graph_bind(g, dev_ws, ws_bytes, stream))


def fsg_graph_stats(g):
    n, nnz, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().fsg_graph_stats(g, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(d)))
    return n.value, nnz.value, d.value


def fsg_graph_destroy(g):
    _check(lib().fsg_graph_destroy(g))


def fsg_default_schedule(g, prm: fsg_params, B) -> fsg_schedule:
    s = fsg_schedule()
    _check(lib().fsg_default_schedule(g, ctypes.byref(prm), B, ctypes.byref(s)))
    return s


def fsg_sim_workspace_size(g, prm: fsg_params, B, sched: Optional[fsg_schedule]) -> int:
    b = ctypes.c_size_t()
    _check(lib().fsg_sim_workspace_size(g, ctypes.byref(prm), B,
                                        ctypes.byref(sched) if sched is not None else None,
                                        ctypes.byref(b)))
    return b.value


def fsg_simulate(g, prm, seeds_addr, n_seeds, B, replicate_offset, rng_key, sched, dev_ws,
                 ws_bytes, states_addr, counts_addr, stream=None) -> fsg_run_info:
    info = fsg_run_info()
    _check(lib().fsg_simulate(g, ctypes.byref(prm), seeds_addr, n_seeds, B, replicate_offset,
                              rng_key & (2**64 - 1),
                              ctypes.byref(sched) if sched is not None else None,
                              dev_ws, ws_bytes, states_addr, counts_addr, ctypes.byref(info),
                              stream))
    return info


def fsg_simulate_noalloc(g, prm, seeds_addr, n_seeds, B, replicate_offset, rng_key, sched,
                         states_addr, counts_addr, stream=None) -> fsg_run_info:
    info = fsg_run_info()
    _check(lib().fsg_simulate_noalloc(g, ctypes.byref(prm), seeds_addr, n_seeds, B,
                                      replicate_offset, rng_key & (2**64 - 1),
                                      ctypes.byref(sched) if sched is not None else None,
                                      states_addr, counts_addr, ctypes.byref(info), stream))
    return info


def fsg_philox4x32_10(dev_ctr, key0, key1, dev_out, count, stream=None):
    _check(lib().fsg_philox4x32_10(dev_ctr, key0, key1, dev_out, count, stream))


def fsg_plan_row_tiles(in_ptr: np.ndarray, heavy: int, row_cost: int, n_parts: int) -> np.ndarray:
    in_ptr = np.ascontiguousarray(in_ptr, dtype=np.int64)
    n = in_ptr.size - 1
    out = np.empty(n + 2, dtype=np.int64)
    cnt = ctypes.c_int64()
    _check(lib().fsg_plan_row_tiles(in_ptr.ctypes.data, n, heavy, row_cost, n_parts,
                                    out.ctypes.data, ctypes.byref(cnt)))
    return out[: cnt.value + 1].copy()


def fsg_batch_plan(jobs_array, n_jobs, steps_per_sync):
    h = ctypes.c_void_p()
    nb = ctypes.c_size_t()
    _check(lib().fsg_batch_plan(jobs_array, n_jobs, steps_per_sync, ctypes.byref(h),
                                ctypes.byref(nb)))
    return h.value, nb.value


def fsg_batch_run(plan, dev_ws, ws_bytes, n_jobs, stream=None):
    infos = (fsg_run_info * n_jobs)()
    total = ctypes.c_double()
    _check(lib().fsg_batch_run(plan, dev_ws, ws_bytes, infos, ctypes.byref(total), stream))
    return list(infos), total.value


def fsg_plan_destroy(plan):
    _check(lib().fsg_plan_destroy(plan))


def fsg_autotune_workspace_size(g, prm, B, batch_only):
    b = ctypes.c_size_t()
    _check(lib().fsg_autotune_workspace_size(g, ctypes.byref(prm), B, int(batch_only),
                                             ctypes.byref(b)))
    return b.value


def fsg_autotune(g, prm, seeds_addr, n_seeds, B, rng_key, tune_steps, batch_only, cache_path,
                 dev_ws, ws_bytes, stream=None):
    best = fsg_schedule()
    bms, dms = ctypes.c_double(), ctypes.c_double()
    _check(lib().fsg_autotune(g, ctypes.byref(prm), seeds_addr, n_seeds, B, rng_key & (2**64 - 1),
                              tune_steps, int(batch_only),
                              cache_path.encode() if cache_path else None, dev_ws, ws_bytes,
                              ctypes.byref(best), ctypes.byref(bms), ctypes.byref(dms), stream))
    return best, bms.value, dms.value


# ---------------------------------------------------- torch-backed helpers --

def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ws(nbytes: int, device):
    import torch
    # +256 so the workspace can be aligned to 256 bytes
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    addr = t.data_ptr()
    return t, (addr + 255) & ~255


def make_params(model, *, p=0.0, ic_prob="uniform", edge_p=None, beta=0.0, gamma=0.0,
                max_steps=-1, alpha=0.0):
    prm = fsg_params()
    prm.model = MODELS[model] if isinstance(model, str) else int(model)
    prm.ic_prob = IC_PROBS[ic_prob] if isinstance(ic_prob, str) else int(ic_prob)
    prm.p = float(p)
    prm.beta = float(beta)
    prm.gamma = float(gamma)
    prm.max_steps = int(max_steps)
    prm.alpha = float(alpha)
    keep = None
    if edge_p is not None:
        keep = np.ascontiguousarray(edge_p, dtype=np.float64)
        prm.edge_p = keep.ctypes.data
    return prm, keep


def make_schedule(d: Optional[dict]) -> Optional[fsg_schedule]:
    if d is None:
        return None
    s = fsg_schedule()
    for k, v in d.items():
        setattr(s, k, int(v))
    return s


class DeviceGraph:
    """A graph bound to device memory owned by a torch tensor; with
    ``out=True`` its out-adjacency too (frontier-driven IC steps)."""

    def __init__(self, ptr, src, device="cuda", out=False):
        ptr = np.ascontiguousarray(ptr, dtype=np.int64)
        src = np.ascontiguousarray(src, dtype=np.int32)
        self.n = ptr.size - 1
        self.nnz = src.size
        self.handle = fsg_graph_create(self.n, self.nnz, ptr.ctypes.data,
                                       src.ctypes.data if src.size else None)
        nbytes = fsg_graph_workspace_size(self.handle)
        self._ws, addr = _ws(nbytes, device)
        fsg_graph_bind(self.handle, addr, nbytes, _stream_ptr())
        self.device = device
        self._out_ws = None
        if out:
            self.bind_out()

    def bind_out(self):
        """Builds the out-adjacency on the device (fsg_graph_bind_out)."""
        nb = _SZ(0)
        _check(lib().fsg_graph_out_workspace_size(self.handle, ctypes.byref(nb)))
        self._out_ws, addr = _ws(nb.value, self.device)
        _check(lib().fsg_graph_bind_out(self.handle, addr, nb.value, _stream_ptr()))

    def stats(self):
        return fsg_graph_stats(self.handle)

    def close(self):
        if self.handle:
            fsg_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation:
    """Workspace and outputs for repeated fsg_simulate calls on one graph.

    The workspace is private to the object and every call uses the same
    graph, parameters, B and schedule, so after a completed run the next
    ones pass FSG_OPT_REUSE_WORKSPACE (the library checks its own tag before
    it leaves buffers uncleared); ``reuse_workspace=False`` turns that off."""

    def __init__(self, graph: DeviceGraph, model, B: int, schedule: Optional[dict] = None,
                 want_states: bool = True, want_counts: bool = True,
                 reuse_workspace: bool = True, **params):
        import torch
        self.graph = graph
        self.B = int(B)
        self.prm, self._keep = make_params(model, **params)
        self.sched = make_schedule(schedule)
        self.reuse_workspace = bool(reuse_workspace)
        self._reuse_sched = make_schedule(dict(schedule or {}))
        self._reuse_sched.options |= OPT_REUSE_WORKSPACE
        self._completed = False
        self.ws_bytes = fsg_sim_workspace_size(graph.handle, self.prm, self.B, self.sched)
        self._ws, self.ws_addr = _ws(self.ws_bytes, graph.device)
        self.states = (torch.empty((graph.n, self.B), dtype=torch.uint8, device=graph.device)
                       if want_states else None)
        self.counts = (torch.empty(graph.n, dtype=torch.int32, device=graph.device)
                       if want_counts else None)

    def run(self, seeds, rng_key: int, replicate_offset: int = 0, stream=None) -> fsg_run_info:
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        sched = self._reuse_sched if (self._completed and self.reuse_workspace) else self.sched
        self._completed = False
        info = fsg_simulate(self.graph.handle, self.prm, seeds.ctypes.data if seeds.size else None,
                            seeds.size, self.B, int(replicate_offset), int(rng_key), sched,
                            self.ws_addr, self.ws_bytes,
                            self.states.data_ptr() if self.states is not None else None,
                            self.counts.data_ptr() if self.counts is not None else None,
                            _stream_ptr(stream))
        self._completed = True
        return info


class Session:
    """fsg_session_*: a run that advances step by step from its current state
    (the paper's run_iteration / run_iterations), with per-step state tallies."""

    def __init__(self, graph: DeviceGraph, model, seeds, B: int, rng_key: int, *,
                 replicate_offset: int = 0, schedule: Optional[dict] = None, stream=None,
                 **params):
        import torch
        self.graph = graph
        self.B = int(B)
        self.prm, self._keep = make_params(model, **params)
        self.sched = make_schedule(schedule)
        self.ws_bytes = fsg_sim_workspace_size(graph.handle, self.prm, self.B, self.sched)
        self._ws, self.ws_addr = _ws(self.ws_bytes, graph.device)
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().fsg_session_begin(graph.handle, ctypes.byref(self.prm),
                                       seeds.ctypes.data if seeds.size else None, seeds.size,
                                       self.B, int(replicate_offset), int(rng_key) & (2**64 - 1),
                                       ctypes.byref(self.sched) if self.sched is not None else None,
                                       self.ws_addr, self.ws_bytes,
                                       _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h.value
        self._torch = torch

    def step(self, n_steps: int = 1, tally: bool = False, stream=None):
        """Advances up to n_steps; returns (fsg_run_info, tally [n_steps, 3] uint64
        numpy array -- pairs in states 1, 2, 3 after each step -- or None)."""
        torch = self._torch
        out = torch.zeros((max(1, int(n_steps)), 3), dtype=torch.int64,
                          device=self.graph.device) if tally else None
        info = fsg_run_info()
        _check(lib().fsg_session_step(self.handle, int(n_steps),
                                      out.data_ptr() if out is not None else None,
                                      ctypes.byref(info), _stream_ptr(stream)))
        return info, (out[:int(n_steps)].cpu().numpy().astype(np.uint64) if tally else None)

    def read(self, want_states: bool = True, stream=None):
        """Current (states [n,B] uint8 tensor or None, counts [n] int32 tensor,
        tally (pairs in states 1, 2, 3))."""
        torch = self._torch
        st = (torch.empty((self.graph.n, self.B), dtype=torch.uint8, device=self.graph.device)
              if want_states else None)
        cnt = torch.empty(self.graph.n, dtype=torch.int32, device=self.graph.device)
        t = torch.zeros(3, dtype=torch.int64, device=self.graph.device)
        _check(lib().fsg_session_read(self.handle, st.data_ptr() if st is not None else None,
                                      cnt.data_ptr(), t.data_ptr(), _stream_ptr(stream)))
        return st, cnt, tuple(int(x) for x in t.cpu().tolist())

    def close(self):
        if getattr(self, "handle", None):
            lib().fsg_session_end(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(graph: DeviceGraph, model, seeds, B, rng_key, *, replicate_offset=0, schedule=None,
             want_states=True, **params):
    """One call: returns (states [n,B] uint8 cuda tensor or None, counts [n] int32 tensor,
    steps_run, absorbed)."""
    sim = Simulation(graph, model, B, schedule=schedule, want_states=want_states, **params)
    info = sim.run(seeds, rng_key, replicate_offset)
    return sim.states, sim.counts, int(info.steps_run), int(info.absorbed)


def fsg_hk_workspace_size(g, B, sched: Optional[fsg_schedule]) -> int:
    out = _SZ(0)
    _check(lib().fsg_hk_workspace_size(g, int(B), ctypes.byref(sched) if sched else None,
                                       ctypes.byref(out)))
    return out.value


def fsg_hk(g, eps, max_steps, B, dev_h, sched, dev_ws, ws_bytes, act, dev_counts,
           stream=None) -> fsg_run_info:
    info = fsg_run_info()
    _check(lib().fsg_hk(g, ctypes.c_float(eps), int(max_steps), int(B), dev_h,
                        ctypes.byref(sched) if sched else None, dev_ws, ws_bytes,
                        ctypes.c_float(act), dev_counts, ctypes.byref(info),
                        stream if stream is not None else _stream_ptr()))
    return info


def fsg_whk(g, eps, mu, max_steps, B, dev_h, sched, dev_ws, ws_bytes, act, dev_counts,
            stream=None) -> fsg_run_info:
    info = fsg_run_info()
    _check(lib().fsg_whk(g, ctypes.c_float(eps), ctypes.c_float(mu), int(max_steps), int(B),
                         dev_h, ctypes.byref(sched) if sched else None, dev_ws, ws_bytes,
                         ctypes.c_float(act), dev_counts, ctypes.byref(info),
                         stream if stream is not None else _stream_ptr()))
    return info


def hk(graph: DeviceGraph, h0, eps: float, max_steps: int, *, act: float = 0.5,
       want_counts: bool = True, schedule=None, mu: float = 1.0):
    """Hegselmann-Krause from opinions h0 ([n, B] float32, any device; copied);
    with mu < 1 the weighted variant (fsg_whk).  Returns (h [n, B] float32 cuda
    tensor, counts [B] int32 tensor of nodes with opinion > act or None,
    fsg_run_info)."""
    import torch
    h = torch.as_tensor(h0, dtype=torch.float32).to(graph.device).contiguous().clone()
    assert h.dim() == 2 and h.shape[0] == graph.n
    B = int(h.shape[1])
    sched = make_schedule(schedule)
    nb = fsg_hk_workspace_size(graph.handle, B, sched)
    ws, addr = _ws(nb, graph.device)
    counts = torch.empty(B, dtype=torch.int32, device=graph.device) if want_counts else None
    info = fsg_whk(graph.handle, float(eps), float(mu), int(max_steps), B, h.data_ptr(), sched,
                   addr, nb, float(act), counts.data_ptr() if counts is not None else None)
    del ws
    return h, counts, info


def autotune(graph: DeviceGraph, model, seeds, B, rng_key, *, tune_steps=None, batch_only=False,
             cache_path=None, **params):
    """Runs the library's autotuner; returns (schedule dict, best ms/step, default ms/step).
    tune_steps None: a window covering the run (the step cap, or 64 steps for runs to
    absorption), since short windows from the seeds time only the run's early phase."""
    prm, keep = make_params(model, **params)
    if tune_steps is None:
        tune_steps = prm.max_steps if prm.max_steps > 0 else 64
    nb = fsg_autotune_workspace_size(graph.handle, prm, int(B), batch_only)
    ws, addr = _ws(nb, graph.device)
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    best, bms, dms = fsg_autotune(graph.handle, prm, seeds.ctypes.data if seeds.size else None,
                                  seeds.size, int(B), int(rng_key), int(tune_steps), batch_only,
                                  cache_path, addr, nb, _stream_ptr())
    del ws, keep
    return best.as_dict(), bms, dms


# Batched steps per captured chunk (one poll of the absorption flags each):
# the batch autotuner chose 8 on the 64-job mixed batch.
BATCH_STEPS_PER_SYNC = 8


class Batch:
    """Several jobs in one batched run (fsg_batch_plan / fsg_batch_run).

    Each job is a dict: graph (DeviceGraph), model, seeds, B, rng_key and
    model parameters, optionally replicate_offset and schedule."""

    PARAM_KEYS = ("p", "ic_prob", "edge_p", "beta", "gamma", "max_steps", "alpha")

    def __init__(self, jobs, steps_per_sync=None, want_states=True, want_counts=True,
                 blocks_per_cu=None):
        import torch
        self.n = len(jobs)
        self._keep = []
        arr = (fsg_job * self.n)()
        self.states, self.counts = [], []
        for i, j in enumerate(jobs):
            g = j["graph"]
            prm, keep = make_params(j["model"], **{k: j[k] for k in self.PARAM_KEYS if k in j})
            seeds = np.ascontiguousarray(j["seeds"], dtype=np.int32)
            self._keep += [keep, seeds]
            st = (torch.empty((g.n, j["B"]), dtype=torch.uint8, device=g.device)
                  if want_states else None)
            ct = torch.empty(g.n, dtype=torch.int32, device=g.device) if want_counts else None
            self.states.append(st)
            self.counts.append(ct)
            a = arr[i]
            a.g = g.handle
            a.prm = prm
            a.seeds = seeds.ctypes.data if seeds.size else None
            a.n_seeds = seeds.size
            a.B = int(j["B"])
            a.replicate_offset = int(j.get("replicate_offset", 0))
            a.rng_key = int(j["rng_key"]) & (2**64 - 1)
            sc = make_schedule(j.get("schedule"))
            if sc is not None:
                a.sched = sc
            a.final_states = st.data_ptr() if st is not None else None
            a.infected_counts = ct.data_ptr() if ct is not None else None
        self._arr = arr
        self.device = jobs[0]["graph"].device
        self.steps_per_sync = int(steps_per_sync or BATCH_STEPS_PER_SYNC)
        self.blocks_per_cu = None
        self.plan, self.ws_bytes = fsg_batch_plan(arr, self.n, self.steps_per_sync)
        if blocks_per_cu is not None:
            self.set_launch(blocks_per_cu)
        self._ws, self.ws_addr = _ws(self.ws_bytes, self.device)

    def set_launch(self, blocks_per_cu: int):
        _check(lib().fsg_batch_set_launch(self.plan, int(blocks_per_cu)))
        self.blocks_per_cu = int(blocks_per_cu)

    def autotune(self, max_trials: int = 32, stream=None):
        """fsg_batch_autotune over this batch; then re-plans with the tuned
        schedules and launch.  Returns a dict of the search's outcome."""
        nb = _SZ(0)
        _check(lib().fsg_batch_autotune_workspace_size(self._arr, self.n, ctypes.byref(nb)))
        ws, addr = _ws(nb.value, self.device)
        tuned = (fsg_job * self.n)()
        sync, bpc, trials = _I32(0), _I32(0), _I32(0)
        bms, dms = ctypes.c_double(0), ctypes.c_double(0)
        _check(lib().fsg_batch_autotune(self._arr, self.n, int(max_trials), addr, nb.value, tuned,
                                        ctypes.byref(sync), ctypes.byref(bpc), ctypes.byref(bms),
                                        ctypes.byref(dms), ctypes.byref(trials), _stream_ptr(stream)))
        del ws
        for i in range(self.n):
            self._arr[i].sched = tuned[i].sched
        fsg_plan_destroy(self.plan)
        self.steps_per_sync = sync.value
        self.plan, self.ws_bytes = fsg_batch_plan(self._arr, self.n, self.steps_per_sync)
        self.set_launch(bpc.value)
        self._ws, self.ws_addr = _ws(self.ws_bytes, self.device)
        return {"best_ms": bms.value, "default_ms": dms.value, "trials": trials.value,
                "steps_per_sync": sync.value, "blocks_per_cu": bpc.value,
                "schedules": [tuned[i].sched.as_dict() for i in range(self.n)]}

    def run(self, stream=None):
        """Returns (list of fsg_run_info, total device ms of the step chunks)."""
        return fsg_batch_run(self.plan, self.ws_addr, self.ws_bytes, self.n, _stream_ptr(stream))

    def close(self):
        if self.plan:
            fsg_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GNN:
    """One member of the surrogate ensemble (fsg_gnn_*): parameters and Adam
    state in a torch device buffer, activations in a per-call workspace."""

    def __init__(self, init_seed: int, device="cuda"):
        import torch
        h = ctypes.c_void_p()
        _check(lib().fsg_gnn_create(64, 3, int(init_seed) & (2**64 - 1), ctypes.byref(h)))
        self.handle = h.value
        cnt = ctypes.c_int64()
        _check(lib().fsg_gnn_param_count(self.handle, ctypes.byref(cnt)))
        self.n_params = cnt.value
        nb = ctypes.c_size_t()
        _check(lib().fsg_gnn_state_size(self.handle, ctypes.byref(nb)))
        self._state, addr = _ws(nb.value, device)
        _check(lib().fsg_gnn_bind(self.handle, addr, nb.value, _stream_ptr()))
        self.device = device
        self._wss = {}

    def _workspace(self, graph: DeviceGraph, n_sets: int):
        key = (graph.handle, n_sets)
        if key not in self._wss:
            nb = ctypes.c_size_t()
            _check(lib().fsg_gnn_workspace_size(self.handle, graph.handle, int(n_sets),
                                                ctypes.byref(nb)))
            t, addr = _ws(nb.value, self.device)
            self._wss = {key: (t, addr, nb.value)}  # keep one workspace at a time
        return self._wss[key]

    def forward(self, graph: DeviceGraph, masks, betas):
        """masks: uint8 cuda tensor [n_sets, n]; betas: sequence of floats.
        Returns probabilities [n_sets, n] (float32 cuda tensor)."""
        import torch
        n_sets = int(masks.shape[0])
        _, addr, nb = self._workspace(graph, n_sets)
        bet = np.ascontiguousarray(betas, dtype=np.float32)
        prob = torch.empty(masks.shape, dtype=torch.float32, device=self.device)
        _check(lib().fsg_gnn_forward(self.handle, graph.handle, n_sets, masks.data_ptr(),
                                     bet.ctypes.data, prob.data_ptr(), addr, nb, _stream_ptr()))
        return prob

    def train_step(self, graph: DeviceGraph, reverse: DeviceGraph, masks, betas, targets,
                   lr: float, update: bool = True) -> float:
        n_sets = int(masks.shape[0])
        _, addr, nb = self._workspace(graph, n_sets)
        bet = np.ascontiguousarray(betas, dtype=np.float32)
        loss = ctypes.c_float()
        _check(lib().fsg_gnn_train_step(self.handle, graph.handle, reverse.handle, n_sets,
                                        masks.data_ptr(), bet.ctypes.data, targets.data_ptr(),
                                        float(lr), int(update), ctypes.byref(loss), addr, nb,
                                        _stream_ptr()))
        return loss.value

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(lib().fsg_gnn_get_params(self.handle, out.ctypes.data, self.n_params, _stream_ptr()))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().fsg_gnn_set_params(self.handle, p.ctypes.data, self.n_params, _stream_ptr()))

    def get_grads(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(lib().fsg_gnn_get_grads(self.handle, out.ctypes.data, self.n_params, _stream_ptr()))
        return out

    def apply_update(self, grads, lr: float):
        """One Adam step with the given gradient (float32 [n_params], host or
        device) or, for None, the last training step's gradient."""
        import torch
        g = None
        if grads is not None:
            g = torch.as_tensor(np.ascontiguousarray(grads, dtype=np.float32)
                                if not isinstance(grads, torch.Tensor) else grads)
            g = g.to(device=self.device, dtype=torch.float32).contiguous()
        _check(lib().fsg_gnn_apply_update(self.handle, g.data_ptr() if g is not None else None,
                                          float(lr), _stream_ptr()))

    def get_state(self):
        """(m, v, BF16 weight copies as uint16, step count)."""
        m = np.empty(self.n_params, dtype=np.float32)
        v = np.empty(self.n_params, dtype=np.float32)
        wb = np.empty(32 * 64 + 2 * 128 * 64, dtype=np.uint16)
        t = ctypes.c_int64()
        _check(lib().fsg_gnn_get_state(self.handle, m.ctypes.data, v.ctypes.data, wb.ctypes.data,
                                       ctypes.byref(t), self.n_params, _stream_ptr()))
        return m, v, wb, t.value

    def close(self):
        if self.handle:
            _check(lib().fsg_gnn_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SpreadEstimator:
    """fsg_estimate_spread: ensemble prediction of the SIR spread, calibrated
    and gated (``gate``: dict with tau, min_seeds, calib), with Monte Carlo
    fallback for queries the gate rejects."""

    def __init__(self, members, graph: DeviceGraph, gamma: float, max_steps: int,
                 B_fallback: int, gate=None, tau=None):
        import torch
        self.members = members
        self.graph = graph
        self.gamma, self.max_steps, self.B = gamma, int(max_steps), int(B_fallback)
        gate = dict(gate or {})
        if tau is not None:
            gate["tau"] = tau
        self.gate = gate
        self._arr = (ctypes.c_void_p * len(members))(*[m.handle for m in members])
        nb = ctypes.c_size_t()
        _check(lib().fsg_gnn_workspace_size(members[0].handle, graph.handle, 1, ctypes.byref(nb)))
        self._ws, self.ws_addr = _ws(nb.value, graph.device)
        self.ws_bytes = nb.value
        prm, _ = make_params("sir", beta=0.5, gamma=gamma, max_steps=max_steps)
        self.sim_bytes = fsg_sim_workspace_size(graph.handle, prm, self.B, None)
        self._sim, self.sim_addr = _ws(self.sim_bytes, graph.device)
        self.counts = torch.empty(graph.n, dtype=torch.int32, device=graph.device)

    def estimate(self, seeds, beta: float, rng_key: int, tau=None):
        """Returns (spread, uncertainty, used_fallback)."""
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        gd = dict(self.gate)
        if tau is not None:
            gd["tau"] = tau
        gate = make_gate(**gd)
        sp, un, fb = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _check(lib().fsg_estimate_spread(self._arr, len(self.members), self.graph.handle,
                                         seeds.ctypes.data if seeds.size else None, seeds.size,
                                         float(beta), float(self.gamma), self.max_steps,
                                         ctypes.byref(gate), self.B,
                                         int(rng_key) & (2**64 - 1), self.ws_addr, self.ws_bytes,
                                         self.sim_addr, self.sim_bytes, self.counts.data_ptr(),
                                         ctypes.byref(sp), ctypes.byref(un), ctypes.byref(fb),
                                         _stream_ptr()))
        return sp.value, un.value, bool(fb.value)
