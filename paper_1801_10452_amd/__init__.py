"""MI355X (gfx950) implementation of the RAPTOR ray-tracing hot path.

The HIP library libraptor_hip.so (built by ``paper_1801_10452_amd.build``) implements the C
ABI of include/raptor.h; ``paper_1801_10452_amd.raptor`` is its Python binding.
"""
from . import raptor  # noqa: F401
