"""MI355X-native WENO5 constrained-transport MHD step (arXiv:1812.04278).

The compute path is the HIP library ``libwenomhd.so`` built from ``csrc/``; the
Python side (:mod:`.binding`) only marshals pointers, sizes and the stream.
Importing the package does not load the library: ``binding`` does, and raises
if it is missing.
"""
__all__ = ["binding", "inputs"]
