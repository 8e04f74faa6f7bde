"""MI355X (gfx950) n-field block solver: GMRES preconditioned by BGS, SIMPLE or
monolithic smoothed-aggregation AMG, all in hand-written HIP kernels behind the
C ABI of include/nfield.h.  This package holds the binding (``nfield``), the
build step (``build``) and the continuous-batching request loop (``serve``)."""
from . import nfield  # noqa: F401
from .nfield import NField, NFieldError  # noqa: F401
