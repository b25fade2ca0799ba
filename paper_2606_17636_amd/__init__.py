"""MI355X spectral-multigrid Poisson solver: HIP library (libsmg.so, C ABI in
include/smg.h) and its ctypes binding."""
from .smg import CYLINDRICAL, SPHERICAL, Batch, Net, Plan, SmgError, load  # noqa: F401
