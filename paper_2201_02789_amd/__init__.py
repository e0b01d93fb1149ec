"""Nested-parallel BFS / SSSP for MI355X (gfx950) with thresholding,
coarsening and multi-block aggregation.

Importing the package loads nothing native.  ``paper_2201_02789_amd.dpo``
is the binding of the HIP library (``libdpo.so``); it raises on first use if
the library is missing.  ``paper_2201_02789_amd.graphgen`` builds inputs.
"""
__all__ = ["dpo", "graphgen"]
