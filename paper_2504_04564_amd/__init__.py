"""MI355X-native compressed-VDB volume sampling and rendering.

The product is ``libvdbc.so`` (C ABI in ``include/vdbc.h``); ``vdbc`` is its
thin Python binding.
"""
from . import vdbc  # noqa: F401

__all__ = ["vdbc"]
