"""ACE build on AMD MI355X: hand-written HIP kernels behind a C ABI (libace.so).

Method: L. Lin, "Adaptively Compressed Exchange Operator", JCTC 2016.
The Python layer only marshals torch device tensors to the C ABI; import
``paper_1601_07159_amd.ace`` for the entry points.
"""
__all__ = ["ace", "synth"]
