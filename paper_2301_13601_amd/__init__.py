"""MI355X-native qubit lattice algorithm (QLA) for the 2D curl-Maxwell
equations in anisotropic dielectric media (arXiv:2301.13601).

Submodules:
  qla     -- Python binding of the HIP library ``libqla.so`` (C ABI in
             include/qla.h): the fused time step, diagnostics and field export.
  scenes  -- seeded synthetic inputs (index profiles, pulses).

Nothing is imported eagerly, so ``scenes`` can be used without the GPU
library being built.
"""

__all__ = ["qla", "scenes"]
