"""FP64 CPU oracle of the differentiable splatting path (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import num_threads, set_num_threads  # noqa: F401
from .ssim import dssim, ssim_map, window_1d  # noqa: F401
from .voxel import downsample, morton_code, voxel_keys  # noqa: F401
