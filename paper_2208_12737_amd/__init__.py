"""MI355X-native Siddon DRR renderer with pose gradients (arXiv:2208.12737).

The computation lives in libdrr.so (HIP kernels for gfx950 behind the C ABI
of include/drr.h); this package holds the ctypes binding, the PyTorch front
end (resident volumes, autograd, NCC loss), batched plans, the request loop
and batched registration.  Importing the package does not load the library;
the first call does, and raises if it is missing.
"""

from .drr import (Detector, Volume, choose_layout, drr, momentum_step, ncc_loss, render, render_backward,
                  render_backward_retrace, render_count, render_l2, render_ncc_grad,
                  render_ncc_loss, render_detector_jacobian)

__all__ = [
    "Detector",
    "Volume",
    "choose_layout",
    "drr",
    "momentum_step",
    "ncc_loss",
    "render",
    "render_backward",
    "render_backward_retrace",
    "render_count",
    "render_l2",
    "render_ncc_grad",
    "render_ncc_loss",
    "render_detector_jacobian",
]
