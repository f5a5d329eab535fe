"""MI355X-native vielbein lattice-Boltzmann hot path (arXiv:1708.05944).

The numerical work runs in ``libvlb.so`` (hand-written HIP for gfx950 behind the C ABI
of ``include/vlb.h``); this package only marshals arguments to it.  There is no CPU
fallback: if the library is missing or no GPU is visible, calls fail loudly.
"""
from .vlb import (VLB_FP64, VLB_MIXED, VLB_TAU_AOKI, VLB_TAU_HYDRO, VLB_TAU_KN, Batch, CouetteDesc, VlbError,  # noqa: F401
                  Channel, ChannelDesc, Mlp, axis_tables, couette_step_noalloc, library_path,
                  load_library, mlp_param_count)

__all__ = ["Batch", "CouetteDesc", "Channel", "ChannelDesc", "Mlp", "mlp_param_count", "VlbError", "axis_tables", "couette_step_noalloc", "load_library", "library_path",
           "VLB_FP64", "VLB_MIXED", "VLB_TAU_AOKI", "VLB_TAU_HYDRO", "VLB_TAU_KN"]
