"""MI355X-native preconditioned s-step CG (Chronopoulos-Gear), after
Bernaschi et al., "Communication-reduced Conjugate Gradient Variants for
GPU-accelerated Clusters" (arXiv 2501.03743).

The solver runs in hand-written HIP kernels for gfx950 behind the C-ABI
library ``libsstep.so`` (declared in ``include/sstep.h``).  ``sstep`` is the
thin ctypes binding; ``workloads`` generates seeded synthetic problems.
Importing the package loads nothing native: the binding loads the library on
first use and raises if it is missing.
"""

__all__ = ["sstep", "workloads"]
