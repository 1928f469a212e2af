"""Binding of the measurement library libmqhpeak (include/mqh_peak.h): reference-kernel rates
that the rooflines' published peaks are checked against.  Not part of the solver."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmqhpeak.so")

MQH_PEAK_COPY = 0
MQH_PEAK_FMA_F32 = 1
MQH_PEAK_FMA_F64 = 2
MQH_PEAK_MFMA_F64 = 3
MQH_PEAK_READ = 4
MQH_PEAK_RSQ_F32 = 5
MQH_PEAK_RSQ_FMA_F32 = 6
MQH_PEAK_MFMA_BF16 = 7


def _load():
    try:
        import torch  # noqa: F401  (one HIP runtime per process, as for the solver library)
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_09798_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.mqh_peak_probe.restype = ctypes.c_int
    L.mqh_peak_probe.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                 ctypes.c_void_p]
    L.mqh_peak_last_error.restype = ctypes.c_char_p
    L.mqh_peak_last_error.argtypes = []
    return L


lib = _load()


def mqh_peak_probe(kind: int, size: int, reps: int = 5, stream=None) -> float:
    """Rate of a reference kernel: bytes/s for MQH_PEAK_COPY and MQH_PEAK_READ, rsq (or rsq + 4 FMA
    groups) per second for MQH_PEAK_RSQ_F32 (MQH_PEAK_RSQ_FMA_F32), flop/s otherwise."""
    rate = ctypes.c_double(0.0)
    st = lib.mqh_peak_probe(int(kind), int(size), int(reps), ctypes.byref(rate),
                            None if stream is None else int(getattr(stream, "cuda_stream", stream)))
    if st != 0:
        raise RuntimeError(f"mqh_peak_probe: status {st} ({lib.mqh_peak_last_error().decode()})")
    return rate.value
