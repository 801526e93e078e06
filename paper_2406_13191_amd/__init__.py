"""MI355X-native projected dual ascent for DCOPF (arXiv 2406.13191).

Submodules:
  synth  - seeded synthetic instances (inputs only)
  _abi   - ctypes binding of the C-ABI library libdcopf_dual.so (HIP kernels)
"""
