"""MI355X-native parallel tempering with isoenergetic cluster moves (arXiv:1501.05630).

`icm` is the ctypes binding of libicm.so (include/icm.h); `inputs` draws the
seeded synthetic workloads.  Nothing here runs the method on the CPU.
"""
from . import inputs  # noqa: F401

__all__ = ["icm", "inputs"]
