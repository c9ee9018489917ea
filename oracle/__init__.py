"""CPU oracle for the hierarchical sparse solver (extended sparsification with
low-rank compression of well-separated fill-in), written in plain FP64
NumPy/SciPy from the paper's definitions.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or run
anything in this package: only the test-suite, the package's smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP path
(kernels, headers, planners, constants); the two meet only at the seeded input
generators, which hold none of the method's arithmetic.

Modules
-------
htree   clusters, adjacency of clusters (Def. "adjacent clusters"), H-tree
        distance (Def. "distance of nodes"), distance-2 colouring of a level
factor  Algorithm 1 (Initialize, MergeRedNodes, Compress, Eliminate)
solve   Algorithms 2-4 (SetRHS, SolveL, SolveU, SplitVar)
gmres   right-preconditioned restarted FGMRES used with the solve as
        preconditioner (Sec. 6.2)

Parity status of each function is stated in its module header.
"""
from .htree import ClusterTree
from .factor import factor, Factorization
from .solve import solve
from .gmres import fgmres

__all__ = ["ClusterTree", "factor", "Factorization", "solve", "fgmres"]
