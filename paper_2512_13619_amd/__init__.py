"""MI355X (gfx950) HDG hot path: batched static condensation, face-block
assembly, preconditioned FGMRES (block-Jacobi, polynomial, Chebyshev) and local
recovery, implemented as HIP kernels in libhdg.so behind the C ABI in
include/hdg.h. `hdg` is the ctypes binding; `pipeline` allocates device
buffers and chains the entry points."""
from . import hdg  # noqa: F401
