"""MI355X-native elastoplastic Newton hot path (arXiv 1805.04155): HIP kernels
behind the C ABI of include/ep.h, with a thin ctypes binding."""
from . import workloads  # noqa: F401
