"""MI355X (gfx950) state-vector gate-application engine.

The hot path (gate classification, fused LDS-tiled passes, on-demand Hadamard
generation, FP64 readouts) runs in the HIP kernels of libsv.so behind the C ABI
of include/sv.h; this package is the thin Python binding on top of it.
"""
from .sv import (GATE_KIND, SVError, StateVector, debug_plan, gate_array,  # noqa: F401
                 lib, last_error)


def __getattr__(name):
    # the torch-facing QNN layer imports torch lazily
    if name in ("QNNFunction", "qnn_expect", "ansatz_gates", "release_cache"):
        from . import qnn
        return getattr(qnn, name)
    raise AttributeError(name)
