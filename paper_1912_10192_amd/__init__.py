"""MI355X-native GRMHD block update (H-AMR method, arxiv 1912.10192).

The compute path lives in the HIP C-ABI library ``libgrmhd.so`` (``csrc/``); the
Python binding in :mod:`paper_1912_10192_amd.grmhd` only marshals arguments.  Importing
this package loads nothing; the library is loaded on first use of the binding.
"""
