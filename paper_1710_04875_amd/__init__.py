"""MI355X-native preconditioned FAS smoothers for the 2-D RANS equations.

The compute path is the HIP library ``libfas.so`` (C ABI in
``include/fas.h``); ``paper_1710_04875_amd.fas`` is its ctypes binding.
Importing this package does not load the library; ``fas.load()`` does,
and raises if it has not been built (``python -m paper_1710_04875_amd.build``).
"""
__all__ = ["fas", "build"]
