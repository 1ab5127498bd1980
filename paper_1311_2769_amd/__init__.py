"""MI355X-native Hough-transform track finder.

The vote and peak search run in hand-written HIP kernels for gfx950 behind
the C ABI declared in include/hough.h (libhough.so, built in-tree by
``python -m paper_1311_2769_amd.build``).  ``hough`` is the Python binding.
"""

__all__ = ["hough"]
