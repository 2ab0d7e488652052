"""Mixture Graph box-histogram queries and transfer-function propagation on MI355X.

- ``Graph``: the Python face of the C ABI in ``include/mg.h`` (libmg.so):
  ``Graph.build`` (CPU factorizer), ``upload``, ``query`` (batched, plain and
  naive GPU kernels), ``footprint``, ``propagate_tf``, ``save`` / ``load``.
- ``synth``: seeded synthetic volumes, boxes and transfer functions.
- ``build_ext``: compiles libmg.so in-tree for gfx950.
"""
from ._lib import MGError, SYMBOLS  # noqa: F401
from .graph import Graph, VARIANTS  # noqa: F401
