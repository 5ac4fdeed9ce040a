"""MI355X-native matrix-free SIPG Helmholtz operator on quad/hex spectral
elements with polynomial non-conforming faces (shared trace space).

The computation lives in the HIP library ``libsipdg.so`` behind the C ABI of
``include/sipdg.h``; this package only marshals arguments.  Importing it
without the built library raises ImportError."""

from ._capi import SipdgError, load as _load_library
from .operator import SipdgOperator, inspect_mesh

_load_library()

__all__ = ["SipdgOperator", "SipdgError", "inspect_mesh"]
