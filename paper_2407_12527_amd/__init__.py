"""MI355X-native random-ordinate-method (ROM) source iteration (arXiv:2407.12527).

The compute path is the C-ABI library ``librom.so`` (hand-written gfx950 HIP kernels, declared
in ``include/rom.h``); ``paper_2407_12527_amd.rom`` is a thin ctypes binding with the same names.
There is no CPU fallback: if the library is missing, loading it raises.
"""
from .rom import *  # noqa: F401,F403
