"""Capture a sequence of libgdm calls on a HIP stream into a hipGraph and
replay it (HIP streams and graphs in place of a tracing compiler).

    g = StreamGraph(stream)            # a non-default torch stream
    g.capture(fn)                      # fn enqueues library calls on `stream`
    g.replay(); g.synchronize()
    g.close()

The library calls inside `fn` must enqueue kernels only (no allocation, host
synchronisation or memset): after gdm_plan, gdm_find_mu with device outputs
(gdm_set_mu_outputs), gdm_subgraph_density_dmu and gdm_mulliken_charges do.
"""
from __future__ import annotations

import ctypes as C

_CAPTURE_RELAXED = 2          # hipStreamCaptureModeRelaxed
_HIP = None


def hip_runtime() -> C.CDLL:
    """The HIP runtime that torch has already loaded (libgdm resolves to the same one)."""
    global _HIP
    if _HIP is None:
        h = C.CDLL("libamdhip64.so.7")
        h.hipStreamBeginCapture.argtypes = [C.c_void_p, C.c_int]
        h.hipStreamEndCapture.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
        h.hipGraphInstantiate.argtypes = [C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_char_p, C.c_size_t]
        h.hipGraphLaunch.argtypes = [C.c_void_p, C.c_void_p]
        h.hipGraphExecDestroy.argtypes = [C.c_void_p]
        h.hipGraphDestroy.argtypes = [C.c_void_p]
        h.hipStreamSynchronize.argtypes = [C.c_void_p]
        _HIP = h
    return _HIP


class StreamGraph:
    def __init__(self, stream):
        self.stream = C.c_void_p(stream.cuda_stream)
        self.hip = hip_runtime()
        self.graph = C.c_void_p()
        self.exe = C.c_void_p()

    def capture(self, fn):
        h = self.hip
        if h.hipStreamBeginCapture(self.stream, _CAPTURE_RELAXED) != 0:
            raise RuntimeError("hipStreamBeginCapture failed")
        try:
            fn()
        finally:
            rc = h.hipStreamEndCapture(self.stream, C.byref(self.graph))
        if rc != 0:
            raise RuntimeError(f"hipStreamEndCapture failed ({rc})")
        if h.hipGraphInstantiate(C.byref(self.exe), self.graph, None, None, 0) != 0:
            raise RuntimeError("hipGraphInstantiate failed")

    def replay(self):
        if self.hip.hipGraphLaunch(self.exe, self.stream) != 0:
            raise RuntimeError("hipGraphLaunch failed")

    def synchronize(self):
        if self.hip.hipStreamSynchronize(self.stream) != 0:
            raise RuntimeError("hipStreamSynchronize failed")

    def close(self):
        if self.exe:
            self.hip.hipGraphExecDestroy(self.exe)
            self.exe = C.c_void_p()
        if self.graph:
            self.hip.hipGraphDestroy(self.graph)
            self.graph = C.c_void_p()
