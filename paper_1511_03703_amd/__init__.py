"""MI355X (gfx950) embedded ensemble propagation for the sampled Q1 diffusion
solve (Phipps et al., arXiv 1511.03703): HIP kernels behind the C ABI of
include/ens.h, bound here with ctypes."""
from . import ens  # noqa: F401
