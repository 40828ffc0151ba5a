"""CPU oracle for recursive skeletonization (Ho & Greengard, "A fast direct solver for
structured linear systems by recursive skeletonization").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 reference written
from the paper.  It may be imported only by the test-suite, by the smoke check of
the package entry point and by the CPU-baseline leg of the benchmark.  The product
(the HIP library and its Python binding) never imports, calls or links it, and it
shares no code with the product: both sides receive their inputs from the
``workloads`` generators only.

Modules
-------
green   Green's functions, Nystrom matrix entries and diagonal rules
tree    quadtree / octree with contiguous index ranges
interp  interpolative decomposition by column-pivoted Householder QR
rs      recursive skeletonization: proxy compression, compressed inverse, solve
dense   brute-force dense matrix and LU solve used to pin the rest

Parity status
-------------
Every function is pinned by tests against closed forms, library reductions or
brute force, except where a docstring says "parity unpinned".
"""
from .green import Problem, KINDS  # noqa: F401
from .tree import Tree, build_tree  # noqa: F401
from .interp import cpqr_id, IDResult  # noqa: F401
from .rs import RSFactor, factor, Options  # noqa: F401
from . import dense  # noqa: F401
