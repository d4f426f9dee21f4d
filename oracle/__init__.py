"""CPU FP64 oracle of the hybrid CNN + Jacobi pressure projection.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct numpy/scipy code
written from the paper (Ajuria Illarramendi, Bauerheim, Cuenot, arXiv
2109.09363): Eq. (2)/(3) and the Jacobi iteration of Sec. 2.2, the
forward-difference divergence of Sec. 3.2, the multi-scale CNN of Sec. 3.1,
the hybrid stop rule of Sec. 3.3 / Sec. 4.1.  Only ``tests/``, the smoke
check of the entry module and the CPU-baseline leg of the benchmark may
import it; the GPU library shares no code with it.

Modules: ``grid`` (planner, D, L, G, E_1), ``solve`` (exact, Jacobi, PCG),
``cnn`` (multi-scale net), ``project`` (one projection), ``advect``
(MacCormack advection + buoyancy), ``adjoint`` (gradient of the
divergence loss).
"""
from . import grid, solve, cnn, project, advect  # noqa: F401
from . import adjoint  # noqa: F401,E402
