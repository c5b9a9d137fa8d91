"""Masked full-batch HMC on MI355X (gfx950).

The sampler draws the selected parameter subset of an MLP or DeepONet from
its conditional posterior with every other parameter fixed (Sec. 3.2,
Algorithm 2 of arXiv 2507.14652).  All compute runs in the HIP library
``libhmc.so`` behind the C ABI of ``include/hmc.h``; ``binding`` marshals
arguments to it.
"""

from .binding import (HMCError, STAT_DTYPE, Sampler, autotune, autotune_workload, load,  # noqa: F401
                      select_mask, sensitivities, trajectory_length)
