"""MI355X-native hot path of strictly single-site DMRG with subspace expansion
(DMRG3S).  The compute lives in the HIP library `libdmrg3s.so` (C-ABI,
declared in include/dmrg3s.h); `paper_1501_05504_amd.abi` is its thin ctypes
binding.  Importing this package does not load the library; importing `abi`
does, and fails loudly when it is not built.
"""
