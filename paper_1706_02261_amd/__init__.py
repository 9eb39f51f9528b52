"""MI355X-native split-step beam propagation (the hot path of biobeam).

Python binding of ``libbpm.so`` (include/bpm.h).  Every step of the march
runs in the library's HIP kernels; this package only checks and marshals
torch tensors (device memory and streams) into the C ABI.
"""
from ._lib import BpmError, lib  # noqa: F401
from .bpm import propagate, workspace_size  # noqa: F401

__all__ = ["BpmError", "lib", "propagate", "workspace_size"]
