"""Python binding of libsv.so (the C ABI in include/sv.h).

Argument marshalling only: every step of gate application runs in the HIP
kernels behind the C ABI. PyTorch provides device memory (the state tensor)
and the HIP stream. If libsv.so is missing, import fails loudly: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_EUNSUPPORTED = 0, -1, -2, -3, -4
SV_C64, SV_C128 = 1, 2

GATE_KIND = {
    "I": 0, "X": 1, "Y": 2, "Z": 3, "H": 4, "S": 5, "SDG": 6, "T": 7, "TDG": 8,
    "RX": 9, "RY": 10, "RZ": 11, "P": 12, "CNOT": 13, "CZ": 14, "SWAP": 15,
    "CPHASE": 16, "MARK": 17, "U1": 18, "U2": 19, "CY": 20, "ISWAP": 21, "DCX": 22,
    "CRZ": 23, "RZZ": 24, "CU1": 25, "CCX": 26, "CSWAP": 27, "SX": 28, "SXDG": 29, "R": 30,
    "U": 31, "RXX": 32, "RYY": 33, "RZX": 34, "ECR": 35, "CH": 36, "CSX": 37, "CU3": 38, "CU": 39,
}
THREE_QUBIT_KINDS = ("CCX", "CSWAP")

OPT_FUSE, OPT_MIN_LOW_QUBITS, OPT_MAX_DENSE, OPT_ON_DEMAND_H, OPT_SMALL_PATH, OPT_PROFILE, OPT_REMAP = \
    1, 2, 3, 4, 5, 6, 7
OPT_PIPELINE = 8

# struct sv_gate (32 bytes)
GATE_DTYPE = np.dtype([("kind", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("param", "<i4"),
                       ("angle", "<f8"), ("index", "<u8")], align=True)
assert GATE_DTYPE.itemsize == 32


class SVError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sv status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        # PyTorch ships its own HIP runtime under the same soname as the
        # system one. Load PyTorch first so that libsv.so binds to the runtime
        # that owns the tensors and streams it is handed; loaded the other way
        # round, the two disagree about devices.
        _torch()
        L = ctypes.CDLL(LIB_PATH)
        P, I, U64, SZ, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
        I64 = ctypes.c_int64
        L.sv_alloc.argtypes = [I, I, I, P, SZ, P, ctypes.POINTER(P)]
        L.sv_free.argtypes = [P]
        L.sv_set_stream.argtypes = [P, P]
        L.sv_set_basis.argtypes = [P, U64]
        L.sv_mark_modified.argtypes = [P]
        L.sv_apply_circuit.argtypes = [P, P, SZ, P, SZ]
        L.sv_expect_z.argtypes = [P, I, P]
        L.sv_norm.argtypes = [P, P]
        L.sv_amplitudes.argtypes = [P, I, P, SZ, P]
        L.sv_expect_z_noalloc.argtypes = [P, I, I, I, I, P, P]
        L.sv_adjoint_expect_z.argtypes = [P, P, SZ, P, SZ, I, P, P]
        L.sv_sync.argtypes = [P]
        L.sv_device_ptr.argtypes = [P]
        L.sv_device_ptr.restype = P
        L.sv_set_option.argtypes = [P, I, I64]
        L.sv_plan_stats.argtypes = [P, P]
        L.sv_profile_read.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I64), ctypes.POINTER(D)]
        L.sv_last_error.restype = ctypes.c_char_p
        L.sv_version.restype = ctypes.c_char_p
        L.sv_debug_plan.argtypes = [I, I, P, SZ, P, SZ, P, P, SZ]
        L.sv_debug_plan.restype = I64
        for name in ("sv_alloc", "sv_free", "sv_set_stream", "sv_set_basis", "sv_apply_circuit",
                     "sv_expect_z", "sv_norm", "sv_amplitudes", "sv_adjoint_expect_z", "sv_sync",
                     "sv_set_option", "sv_plan_stats", "sv_profile_read", "sv_mark_modified",
                     "sv_expect_z_noalloc"):
            getattr(L, name).restype = I
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != SV_OK:
        raise SVError(status, lib().sv_last_error().decode())


def last_error() -> str:
    return lib().sv_last_error().decode()


def gate_array(gates: Sequence) -> np.ndarray:
    """Gate records (objects with name, q0, q1, angle, param, index and, for
    CCX / CSWAP, q2) -> sv_gate[] (a 3-qubit gate's q2 goes in `index`)."""
    arr = np.zeros(len(gates), dtype=GATE_DTYPE)
    for i, g in enumerate(gates):
        idx = g.q2 if g.name in THREE_QUBIT_KINDS else g.index
        arr[i] = (GATE_KIND[g.name], g.q0, g.q1, g.param, g.angle, idx)
    return arr


def expect_z_noalloc(state, n: int, qubit: int, out, stream=None, batch: Optional[int] = None) -> None:
    """<Z_qubit> (qubit >= 0) or the norm (qubit = -1) of the states in the
    device tensor `state` ([batch, 2^n], complex64 or complex128) into the
    device tensor `out` (float64, [batch]), asynchronously on `stream` (a
    torch.cuda.Stream; default: the current stream), with no allocation."""
    torch = _torch()
    if state.dtype not in (torch.complex64, torch.complex128) or not state.is_contiguous():
        raise ValueError("state must be a contiguous complex64 or complex128 tensor")
    if out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor")
    b = state.numel() >> n if batch is None else int(batch)
    if out.numel() < b or state.numel() < (b << n):
        raise ValueError("state or out is smaller than batch * 2^n")
    st = stream if stream is not None else torch.cuda.current_stream(state.device)
    dt = SV_C128 if state.dtype == torch.complex128 else SV_C64
    _check(lib().sv_expect_z_noalloc(ctypes.c_void_p(state.data_ptr()), int(n), dt, b, int(qubit),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream)))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _torch():
    import torch
    return torch


class StateVector:
    """A batch of n-qubit states in HBM, held by a torch tensor [batch, 2^n].

    dtype: "c128" (torch.complex128) or "c64" (torch.complex64).
    stream: a torch.cuda.Stream (default: the current stream at creation).
    """

    def __init__(self, n: int, dtype: str = "c128", batch: int = 1, device=None, stream=None):
        torch = _torch()
        if dtype not in ("c128", "c64"):
            raise ValueError("dtype must be 'c128' or 'c64'")
        self.n = int(n)
        self.batch = int(batch)
        self.dtype = dtype
        tdt = torch.complex128 if dtype == "c128" else torch.complex64
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.tensor = torch.empty((self.batch, 1 << self.n), dtype=tdt, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        nbytes = self.tensor.numel() * self.tensor.element_size()
        _check(lib().sv_alloc(self.n, SV_C128 if dtype == "c128" else SV_C64, self.batch,
                              ctypes.c_void_p(self.tensor.data_ptr()), nbytes,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    # -- lifetime -------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().sv_free(self._h))
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

    @property
    def handle(self):
        return self._h

    # -- operations -----------------------------------------------------------
    def set_basis(self, j: int) -> None:
        _check(lib().sv_set_basis(self._h, int(j)))

    def load(self, values) -> None:
        """Copy host amplitudes [batch, 2^n] (or [2^n]) into the state."""
        torch = _torch()
        src = torch.as_tensor(np.asarray(values).reshape(self.batch, -1)).to(self.tensor.dtype)
        with torch.cuda.stream(self.stream):
            self.tensor.copy_(src.to(self.tensor.device, non_blocking=False))
        _check(lib().sv_mark_modified(self._h))

    def mark_modified(self) -> None:
        _check(lib().sv_mark_modified(self._h))

    def apply(self, gates, params: Optional[np.ndarray] = None) -> None:
        """Apply a gate list (synth.Gate records or an sv_gate array)."""
        arr = gates if isinstance(gates, np.ndarray) and gates.dtype == GATE_DTYPE else gate_array(gates)
        arr = np.ascontiguousarray(arr)
        p = None
        n_params = 0
        if params is not None:
            p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(self.batch, -1))
            n_params = p.shape[1]
        _check(lib().sv_apply_circuit(self._h, _ptr(arr), len(arr), _ptr(p), n_params))

    def expect_z(self, qubit: int) -> np.ndarray:
        out = np.zeros(self.batch, dtype=np.float64)
        _check(lib().sv_expect_z(self._h, int(qubit), _ptr(out)))
        return out

    def norm(self) -> np.ndarray:
        out = np.zeros(self.batch, dtype=np.float64)
        _check(lib().sv_norm(self._h, _ptr(out)))
        return out

    def amplitudes(self, idx: Iterable[int], b: int = 0) -> np.ndarray:
        ix = np.ascontiguousarray(np.asarray(list(idx) if not isinstance(idx, np.ndarray) else idx,
                                             dtype=np.uint64))
        out = np.zeros(2 * len(ix), dtype=np.float64)
        _check(lib().sv_amplitudes(self._h, int(b), _ptr(ix), len(ix), _ptr(out)))
        return out[0::2] + 1j * out[1::2]

    def adjoint_expect_z(self, gates, params: np.ndarray, qubit: int = 0):
        arr = gates if isinstance(gates, np.ndarray) and gates.dtype == GATE_DTYPE else gate_array(gates)
        arr = np.ascontiguousarray(arr)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(self.batch, -1))
        expect = np.zeros(self.batch, dtype=np.float64)
        grad = np.zeros(p.shape, dtype=np.float64)
        _check(lib().sv_adjoint_expect_z(self._h, _ptr(arr), len(arr), _ptr(p), p.shape[1],
                                         int(qubit), _ptr(expect), _ptr(grad)))
        return expect, grad

    def sync(self) -> None:
        _check(lib().sv_sync(self._h))

    def set_option(self, option: int, value: int) -> None:
        _check(lib().sv_set_option(self._h, int(option), int(value)))

    def plan_stats(self) -> dict:
        out = np.zeros(8, dtype=np.int64)
        _check(lib().sv_plan_stats(self._h, _ptr(out)))
        keys = ("passes", "exchanges", "gates", "generated_h", "launches", "hbm_bytes", "relabels",
                "generated_product")
        return {k: int(out[i]) for i, k in enumerate(keys)}

    def profile_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        by = ctypes.c_double()
        _check(lib().sv_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
        return ms.value, n.value, by.value

    def numpy(self) -> np.ndarray:
        self.sync()
        return self.tensor.detach().cpu().numpy()


PASS_DTYPE = np.dtype([("k", "<i4"), ("w", "<i4"), ("op_begin", "<i4"), ("op_end", "<i4"),
                       ("layout_begin", "<i4"), ("flags", "<u4"), ("tiles", "<u8"),
                       ("gen_j", "<u8"), ("gen_mask", "<u8"), ("gen_scale", "<f8"),
                       ("store_layout", "<i4"), ("q", "u1", (28,)), ("n_layouts", "<i4"),
                       ("pad", "u1", (4,))])
LAYOUT_DTYPE = np.dtype([("thr_goff", "<u8", (10,)), ("reg_goff", "<u8", (6,)),
                         ("goff_xor", "<u8"), ("reg_goff_xor", "<u8"),
                         ("thr_slot", "<u4", (10,)), ("reg_slot", "<u4", (6,)),
                         ("slot_xor", "<u4"), ("flags", "<u4"), ("xor_local", "<u4"),
                         ("thr_local", "u1", (10,)), ("reg_local", "u1", (6,)),
                         ("pad", "u1", (20,))])
assert LAYOUT_DTYPE.itemsize == 256
OP_DTYPE = np.dtype([("code", "u1"), ("a", "u1"), ("b", "u1"), ("sa", "u1"), ("sb", "u1"),
                     ("pad", "u1", (3,)), ("data", "<u8"), ("payload", "<f8", (8,))])
SOP_DTYPE = np.dtype([("code", "u1"), ("q0", "u1"), ("q1", "u1"), ("q2", "u1"), ("pad", "u1", (4,)),
                      ("data", "<u8")])
assert PASS_DTYPE.itemsize == 96 and LAYOUT_DTYPE.itemsize == 256
assert OP_DTYPE.itemsize == 80 and SOP_DTYPE.itemsize == 16


def debug_plan(n: int, gates, dtype: str = "c128", params: Optional[np.ndarray] = None,
               fuse: bool = True, min_low: int = 6, max_dense: int = 1 << 20,
               gen_h: bool = True, basis: Optional[int] = 0, small_mode: int = 1,
               remap: bool = True, basis_in_memory: bool = True) -> dict:
    """The plan sv_apply_circuit would run (no GPU needed): see include/sv_debug.h."""
    arr = np.ascontiguousarray(gate_array(gates))
    p = None if params is None else np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
    opts = np.array([int(fuse), min_low, max_dense, int(gen_h), int(basis is not None),
                     0 if basis is None else basis, small_mode, int(remap),
                     int(basis is not None and not basis_in_memory)], dtype=np.int64)
    dt = SV_C128 if dtype == "c128" else SV_C64
    L = lib()
    need = L.sv_debug_plan(n, dt, _ptr(arr), len(arr), _ptr(p), 0 if p is None else len(p),
                           _ptr(opts), None, 0)
    if need < 0:
        raise SVError(int(need), last_error())
    buf = np.zeros(int(need), dtype=np.uint8)
    got = L.sv_debug_plan(n, dt, _ptr(arr), len(arr), _ptr(p), 0 if p is None else len(p),
                          _ptr(opts), _ptr(buf), len(buf))
    if got != need:
        raise SVError(SV_EINVAL, "debug plan size changed")
    h = buf[:256].view(np.int64)
    out = {"small": bool(h[0]), "k": int(h[9]), "w": int(h[10]), "R": int(h[11]), "m": int(h[12]),
           "exchanges": int(h[6]), "generated_h": int(h[7]), "gates": int(h[8]),
           "hbm_bytes": int(h[18]), "cstride": int(h[5]), "relabels": int(h[19]), "restores": int(h[20]),
           "min_low": int(h[21]), "generated_product": int(h[22])}

    def take(off, count, dt_):
        return buf[off: off + count * dt_.itemsize].view(dt_).copy()

    out["passes"] = take(int(h[13]), int(h[1]), PASS_DTYPE)
    out["layouts"] = take(int(h[14]), int(h[2]), LAYOUT_DTYPE)
    out["ops"] = take(int(h[15]), int(h[3]), OP_DTYPE)
    out["sops"] = take(int(h[16]), int(h[4]), SOP_DTYPE)
    # constants and op payloads are in the state's precision
    f32 = dtype == "c64"
    rb = 4 if f32 else 8
    out["f32"] = f32
    out["consts"] = buf[int(h[17]): int(h[17]) + rb * int(h[5])].view(
        np.float32 if f32 else np.float64).astype(np.float64)
    return out
