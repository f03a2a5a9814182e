"""Dead-time Markov stationary PDFs for asynchronous single-photon LiDAR on
MI355X (gfx950): HIP kernels behind the C-ABI of include/dtm.h, with a thin
ctypes binding in ``paper_2509_20500_amd.dtm``."""
from . import dtm  # noqa: F401
