"""MI355X-native LBM-IBM (D3Q19 BGK + multi-direct-forcing immersed boundary).

The compute path lives in the HIP library ``liblbmibm.so`` built from
``csrc/``; ``lbmibm`` is its thin ctypes binding.  Importing the package does
not load the library; ``paper_1904_02108_amd.lbmibm`` does, and fails loudly
when it has not been built.
"""
__all__ = ["lbmibm", "workload"]
