"""MI355X-native CLAK-Eig: the multi-trait GWAS grid of GLS problems on gfx950.

The compute path is the HIP library ``_lib/libclak.so`` behind the C ABI of
``include/clak.h``; :mod:`paper_1207_2169_amd.clak` is a thin ctypes binding
with the same function names.  PyTorch only provides device memory and
streams.
"""
from . import clak  # noqa: F401
from .clak import ClakError  # noqa: F401
