"""MI355X (gfx950) semi-Lagrangian MGRIT for periodic linear advection
(De Sterck, Falgout & Krzysik, arXiv 2203.13382).

The compute path is the HIP library ``libslmgrit.so`` behind the C ABI of
``include/slmgrit.h``; ``Plan`` (one problem) and ``Batch`` (many 1D problems) are thin
bindings over it.
"""
from .plan import Batch, Plan  # noqa: F401
from .workloads import Problem, Solver, config  # noqa: F401
