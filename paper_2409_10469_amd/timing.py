"""Stream timing events for the measurements.

HIP events are recorded here with a device-scope release (hipEventReleaseToDevice).
An event recorded with the default system-scope release writes the L2 cache back to
memory when it completes. Placed between two kernels, it holds back the second kernel
by that write-back, several microseconds after a rollout that leaves megabytes of noise
in the L2, and the second kernel then misses in the L2. The timestamps are the same
either way. Read an event only after the stream has been synchronised.
"""
import ctypes as C

_HIP_EVENT_RELEASE_TO_DEVICE = 0x40000000
_hip = None


def _runtime():
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (loads the HIP runtime that torch and the library share)
        h = C.CDLL("libamdhip64.so.7")
        h.hipEventCreateWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_uint]
        h.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
        h.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        h.hipEventDestroy.argtypes = [C.c_void_p]
        _hip = h
    return _hip


class DeviceEvent:
    """A timing event on a torch stream (the current one when none is given)."""

    def __init__(self):
        self._h = C.c_void_p()
        rc = _runtime().hipEventCreateWithFlags(C.byref(self._h), _HIP_EVENT_RELEASE_TO_DEVICE)
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")

    def record(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = _runtime().hipEventRecord(self._h, C.c_void_p(s.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def elapsed_time(self, end):
        """Milliseconds from this event to `end` (both recorded and complete)."""
        ms = C.c_float()
        rc = _runtime().hipEventElapsedTime(C.byref(ms), self._h, end._h)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return ms.value

    def __del__(self):
        if getattr(self, "_h", None) and _hip is not None:
            _hip.hipEventDestroy(self._h)
            self._h = None
