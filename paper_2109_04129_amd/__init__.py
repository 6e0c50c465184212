"""MI355X-native H-matrix power-series EFIE solver (arXiv:2109.04129).

The compute path is the C-ABI library ``libhps.so`` (host C++ for the
H-matrix build and the symbolic setup, HIP kernels for gfx950 for the
scaling-coefficient setup and the power-series solve).  ``hps`` is a thin
ctypes binding with the same function names as ``include/hps.h``.
"""

from . import hps  # noqa: F401
