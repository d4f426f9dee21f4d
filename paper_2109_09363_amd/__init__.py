"""hyproj: hybrid CNN + Jacobi pressure projection on a 2D MAC grid for
MI355X (gfx950).  The projection runs in the HIP library libhyproj.so
(C ABI in include/hyproj.h); this package is its thin Python binding."""
from .api import Batch, Projector, ProjectionResult, ProjectionLoss, adam_async, project  # noqa: F401
from ._lib import HypError, lib  # noqa: F401
