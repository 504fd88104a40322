"""MI355X-native explicit spectral-cell wave solver (immersed boundary, central
differences).  ``fcw`` is the ctypes binding of the C ABI in include/fcw.h; ``solver``
wraps it with torch device buffers and streams."""
from . import fcw  # noqa: F401

__all__ = ["fcw"]
