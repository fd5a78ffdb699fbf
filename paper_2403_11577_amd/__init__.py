"""MI355X-native differentiable Gaussian-splatting path of 3DGS-Calib (arXiv 2403.11577).

``binding``  -- ctypes mirror of include/splat.h (argument marshalling only);
``pipeline`` -- device buffers, the batched step and the per-view plain driver,
                the autograd Function, hipGraph capture and the autotuner.

Nothing is imported eagerly, so the synthetic-input module and the oracle can be
used without loading the HIP library.
"""
__all__ = ["binding", "pipeline", "build"]
