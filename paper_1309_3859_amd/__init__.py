"""MI355X-native hot path of the compact U(1) Luscher--Weisz multilevel method
(Amado, Cardoso, Bicudo, arXiv 1309.3859): checkerboard heatbath and
overrelaxation inside frozen-boundary time slabs, slab-averaged two-link and
plaquette-insertion operators, and their products into Polyakov-loop
correlators and flux-tube field profiles.

The compute path is libu1ml.so (HIP, gfx950) behind the C ABI in
include/u1ml.h; ``u1ml`` is its Python binding, ``configs`` the workload
presets and ``analysis`` the host-side estimators.
"""
from . import configs  # noqa: F401

__all__ = ["configs", "u1ml", "analysis", "build"]
