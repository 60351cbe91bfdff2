"""MI355X (gfx950) lattice-QCD Dirac operators and solvers.

The computation lives in the HIP library ``liblqcd.so`` (C ABI:
include/lqcd.h); ``lqcd`` is its ctypes binding under the same names and
``ops`` builds operator instances on the GPU.
"""
from . import lqcd  # noqa: F401
