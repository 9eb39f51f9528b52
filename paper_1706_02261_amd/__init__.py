"""MI355X-native split-step beam propagation (the hot path of biobeam).

Python binding of ``libbpm.so`` (include/bpm.h).  Every step of the march
runs in the library's HIP kernels; this package only checks and marshals
torch tensors (device memory and streams) into the C ABI.
"""
from ._lib import BpmError, lib  # noqa: F401
from .bpm import (BPMFunction, PreparedBatch, PupilBPMFunction, adam_step, adjoint,  # noqa: F401
                  adjoint_batch,
                  fft2, guide_star_phase, march_phase_times, point_sources, propagate, propagate_adapted,
                  propagate_batch, psf_readout, slice_means,
                  pupil_phase_grad, pupil_spectrum, set_wait_limit, workspace,
                  workspace_size, workspace_status)

__all__ = ["BpmError", "lib", "propagate", "propagate_batch", "PreparedBatch", "adjoint", "fft2",
           "pupil_spectrum", "pupil_phase_grad", "psf_readout", "point_sources", "BPMFunction",
           "PupilBPMFunction", "workspace", "workspace_size", "workspace_status",
           "set_wait_limit", "march_phase_times", "propagate_adapted", "slice_means",
           "guide_star_phase", "adam_step", "adjoint_batch"]
