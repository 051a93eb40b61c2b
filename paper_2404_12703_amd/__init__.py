"""MI355X (gfx950) DGSEM Navier-Stokes hot path: a HIP library behind a C ABI
(include/dgsem.h) with a thin ctypes binding.  See binding.Solver / binding.Server."""
from .binding import (DGError, Server, Solver, lib, workspace_bytes,  # noqa: F401
                      REQ_DONE, REQ_FAILED, REQ_QUEUED, REQ_RUNNING)
