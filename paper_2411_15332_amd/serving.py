"""Serving: Python side of the continuous-batching engine (sv_engine_* in include/sv.h).

ServingEngine marshals requests to the C++ scheduler in libsv.so; every state
update and readout runs in the gfx950 kernels. run_stream() replays a timed
arrival stream against an engine and records per-request latency from the
scheduled arrival time to the moment the result is back on the host.
"""
from __future__ import annotations

import ctypes
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

from .sv import GATE_DTYPE, SV_C64, SV_C128, _check, _ptr, gate_array, lib


def _engine_lib():
    L = lib()
    if not getattr(L, "_engine_ready", False):
        P, I, U64, SZ, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int64
        L.sv_engine_create.argtypes = [I, I, I, SZ, ctypes.POINTER(P)]
        L.sv_engine_create_stepped.argtypes = [I, I, I, I, SZ, ctypes.POINTER(P)]
        L.sv_engine_free.argtypes = [P]
        L.sv_engine_submit.argtypes = [P, U64, I, P, SZ, P, SZ, I]
        L.sv_engine_poll.argtypes = [P, I64, P, P, SZ, ctypes.POINTER(SZ)]
        L.sv_engine_stats.argtypes = [P, P]
        L.sv_engine_register.argtypes = [P, I, P, SZ, SZ, I, ctypes.POINTER(I64)]
        L.sv_engine_submit_registered.argtypes = [P, U64, I64, P, SZ]
        for name in ("sv_engine_create", "sv_engine_create_stepped", "sv_engine_free", "sv_engine_submit",
                     "sv_engine_poll", "sv_engine_stats", "sv_engine_register", "sv_engine_submit_registered"):
            getattr(L, name).restype = I
        L._engine_ready = True
    return L


class ServingEngine:
    """dtype "c64" or "c128"; max_batch requests per launch group; n_streams
    groups in flight; hbm_budget_bytes of state memory (0: unlimited).
    stepped=True: continuous batching at pass granularity for the larger
    states (sv_engine_create_stepped), with at most max_active of them on the
    GPU; max_batch and n_streams then apply to the small states."""

    def __init__(self, dtype: str = "c64", max_batch: int = 256, n_streams: int = 4,
                 hbm_budget_bytes: int = 0, stepped: bool = False, max_active: int = 256):
        self.L = _engine_lib()
        h = ctypes.c_void_p()
        dt = SV_C64 if dtype == "c64" else SV_C128
        if stepped:
            _check(self.L.sv_engine_create_stepped(dt, int(max_active), int(max_batch), int(n_streams),
                                                   int(hbm_budget_bytes), ctypes.byref(h)))
        else:
            _check(self.L.sv_engine_create(dt, int(max_batch), int(n_streams), int(hbm_budget_bytes),
                                           ctypes.byref(h)))
        self._h = h
        self.dtype = dtype
        self._ids = np.zeros(4096, dtype=np.uint64)
        self._vals = np.zeros(4096, dtype=np.float64)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(self.L.sv_engine_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, rid: int, n: int, gates, params: Optional[np.ndarray] = None, qubit: int = 0) -> None:
        arr = gates if isinstance(gates, np.ndarray) and gates.dtype == GATE_DTYPE else gate_array(gates)
        arr = np.ascontiguousarray(arr)
        p = None if params is None else np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
        _check(self.L.sv_engine_submit(self._h, int(rid), int(n), _ptr(arr), len(arr), _ptr(p),
                                       0 if p is None else len(p), int(qubit)))

    def register(self, n: int, gates, n_params: int, qubit: int = 0) -> int:
        """Plan a circuit once; returns its handle for submit_registered."""
        arr = gates if isinstance(gates, np.ndarray) and gates.dtype == GATE_DTYPE else gate_array(gates)
        arr = np.ascontiguousarray(arr)
        cid = ctypes.c_int64()
        _check(self.L.sv_engine_register(self._h, int(n), _ptr(arr), len(arr), int(n_params), int(qubit),
                                         ctypes.byref(cid)))
        return cid.value

    def submit_registered(self, rid: int, circuit: int, params: np.ndarray) -> None:
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
        _check(self.L.sv_engine_submit_registered(self._h, int(rid), int(circuit), _ptr(p), len(p)))

    def poll(self, wait_us: int = 0) -> List[Tuple[int, float]]:
        cnt = ctypes.c_size_t()
        _check(self.L.sv_engine_poll(self._h, int(wait_us), _ptr(self._ids), _ptr(self._vals),
                                     len(self._ids), ctypes.byref(cnt)))
        c = cnt.value
        return list(zip(self._ids[:c].tolist(), self._vals[:c].tolist()))

    def stats(self) -> Dict[str, int]:
        out = np.zeros(8, dtype=np.int64)
        _check(self.L.sv_engine_stats(self._h, _ptr(out)))
        keys = ("queued", "in_flight", "completed", "groups", "state_bytes", "largest_group",
                "deferred", "small_groups")
        return {k: int(out[i]) for i, k in enumerate(keys)}


def run_stream(engine: ServingEngine, requests: Sequence, gates_of, rate_scale: float = 1.0,
               timeout_s: float = 120.0, key_of=None) -> Dict[str, object]:
    """Replay ``requests`` (objects with rid, arrival_s, n, params) against the
    engine in real time: request r is submitted when the clock passes
    r.arrival_s * rate_scale. gates_of(r) gives its sv_gate array; with
    key_of(r) (a hashable circuit key), each distinct circuit is registered
    once and requests are submitted by handle.
    Returns per-request latency (s) and result, plus the wall time."""
    cids: Dict[object, int] = {}

    def submit(r):
        if key_of is None:
            engine.submit(r.rid, r.n, gates_of(r), r.params, 0)
            return
        k = key_of(r)
        cid = cids.get(k)
        if cid is None:
            cid = cids[k] = engine.register(r.n, gates_of(r), len(r.params), 0)
        engine.submit_registered(r.rid, cid, r.params)

    order = sorted(requests, key=lambda r: r.arrival_s)
    arrival = {r.rid: r.arrival_s * rate_scale for r in order}
    done: Dict[int, Tuple[float, float]] = {}
    t0 = time.perf_counter()
    i = 0
    while len(done) < len(order):
        now = time.perf_counter() - t0
        if now > timeout_s:
            raise TimeoutError(f"stream did not drain in {timeout_s} s ({len(done)}/{len(order)})")
        while i < len(order) and arrival[order[i].rid] <= now:
            submit(order[i])
            i += 1
        nxt = arrival[order[i].rid] - now if i < len(order) else 1e9
        wait = int(max(0.0, min(nxt, 0.002)) * 1e6)
        for rid, val in engine.poll(wait_us=wait):
            done[rid] = (time.perf_counter() - t0 - arrival[rid], val)
    wall = time.perf_counter() - t0
    lat = np.array([done[r.rid][0] for r in order])
    return {"latency_s": lat, "values": {rid: v for rid, (_, v) in done.items()}, "wall_s": wall,
            "first_arrival_s": arrival[order[0].rid], "last_arrival_s": arrival[order[-1].rid]}


def summarize(res: Dict[str, object], count: int, warmup: int = 0) -> Dict[str, float]:
    lat = np.asarray(res["latency_s"])[warmup:]
    span = res["wall_s"] - res["first_arrival_s"]
    return {"circuits_per_s": count / span if span > 0 else float("nan"),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "requests": int(count)}
