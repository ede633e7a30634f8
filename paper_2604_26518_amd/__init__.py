"""MI355X periodic geometric-multigrid homogenization (libgmt) -- Python side.

The compute path lives in ``libgmt.so`` (HIP, gfx950) behind the C ABI of
``include/gmt.h``; ``binding`` only marshals arguments.  Import
``paper_2604_26518_amd.binding`` for the ``Hierarchy`` class.
"""

__all__ = ["binding", "build"]
