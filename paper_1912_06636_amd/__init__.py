"""MI355X-native real-space grid engine for numeric atom-centred orbitals.

The library is libnao.so (include/nao.h); ``paper_1912_06636_amd.nao`` is its thin
ctypes binding.  Build with ``python -m paper_1912_06636_amd.build``.
"""
