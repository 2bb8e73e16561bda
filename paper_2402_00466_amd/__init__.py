"""MI355X (gfx950) mEVP momentum subcycle of the neXtSIM-DG dynamical core.

``libmevp.so`` (HIP kernels + C ABI, see include/mevp.h) does all the work;
``paper_2402_00466_amd.mevp`` is the ctypes binding with torch tensors for
device memory and streams.
"""
from .mevp import (Context, Domain, MevpError, Params, default_params, lib, lib_path,
                   step_static, workspace_size, EXPORTS, FP64, MIXED, STATIC_SCRATCH_BYTES,
                   STRATEGIES, TILES)

__all__ = ["Context", "Domain", "MevpError", "Params", "default_params", "lib", "lib_path",
           "step_static", "workspace_size", "EXPORTS", "FP64", "MIXED", "STATIC_SCRATCH_BYTES",
           "STRATEGIES", "TILES"]
