"""MI355X (gfx950) implementation of ATSFFT, the adaptive-tuning sparse FFT
(Shi, Yang, Zhang, You; arXiv:1908.02461).  The transform runs in the HIP
library libatsfft.so behind the C ABI of include/atsfft.h; ``atsfft`` is its
Python binding."""

__version__ = "0.1.0"
