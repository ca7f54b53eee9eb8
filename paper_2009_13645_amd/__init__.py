"""MI355X-native boosted-frame FDTD/PIC step of the MITHRA 2.0 FEL method.

The compute path lives in the HIP library built from `csrc/`; the Python
layer in `engine.py` only marshals arguments through its C ABI.  Nothing is
imported eagerly here, so `workloads` can be used without the library.
"""
__all__ = ["engine", "workloads"]
