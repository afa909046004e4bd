"""MI355X-native D3Q27 central-moment lattice Boltzmann step with immersed
boundary coupling (arXiv:2101.11856), behind the C-ABI library ``liblbm``.

Submodules:
  lbm    -- ctypes binding of ``include/lbm.h`` (loads ``liblbm.so``; fails
            loudly if it is missing)
  synth  -- seeded synthetic inputs (flow fields, solid samples); numpy only
  adjoint -- torch.autograd.Function around the forward/adjoint entry points
"""
__all__ = ["lbm", "synth"]
