"""MI355X-native GRPIC particle push + deposit (arXiv:2503.04558 hot path).

The compute path is the HIP library ``libgrpic.so`` behind the C ABI declared
in ``include/grpic.h``; ``paper_2503_04558_amd.grpic`` is its ctypes binding.
Submodules are imported on demand so that the input generator can be used on
machines without the built library.
"""
