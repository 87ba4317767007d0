"""MI355X-native TO-LRS lattice Boltzmann LES (HIP kernels for gfx950 behind a C ABI).

The compute path is ``liblbm_hip.so`` (``csrc/``, declared in ``include/lbm.h``);
``lbm`` is its ctypes binding.  Build with ``paper_2609_32892_amd.build.build()``.
"""
from .lbm import (  # noqa: F401
    BGK, D2Q9, D3Q19, FP32_PLAIN, FP32_SHIFTED, FP64, FORCE_CONST_X, FORCE_NONE, FORCE_SIN_Y,
    SMAGORINSKY, WALE, Batch, ClosureSpec, LbmError, Run, lattice_info, lib, make_config,
)
