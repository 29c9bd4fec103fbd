"""MI355X-native focused-transport pseudo-particle path (HIP kernels behind a C ABI).

The product is ``libfte.so`` (``csrc/``, declared in ``include/fte.h``); the
binding in ``fte.py`` only marshals arguments.  Build with
``python -m paper_2404_12164_amd.build``.
"""
from . import fte  # noqa: F401
