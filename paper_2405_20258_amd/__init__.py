"""Static-subspace RPA correlation energies on AMD MI355X (gfx950).

The compute path is the HIP library libssrpa.so (C ABI in include/ssrpa.h);
`ssrpa` is its ctypes binding.  Importing the binding fails loudly when the
library has not been built.
"""
__all__ = ["ssrpa"]
