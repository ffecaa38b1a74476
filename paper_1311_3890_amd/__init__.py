"""MI355X-native TB-SMA molecular dynamics of gold nanowires under elongation.

The compute path is libtbsma.so (HIP for gfx950, C ABI in include/tbsma.h);
this package holds its build script, a ctypes binding and ``WireBatch``, which
lays replicas out in device memory and forwards each operation to the
library.
"""
from ._abi import TbsmaError, lib  # noqa: F401
from .engine import MASS_AU, Potential, WireBatch, build_wire_host  # noqa: F401
