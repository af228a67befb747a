"""MI355X (gfx950) hot path of DMTS-NC: distilled multi-time-stepping with
non-conservative forces (arXiv 2602.14975).

The computation lives in the HIP library ``libnnp.so`` (C interface in
``include/nnp.h``); this package is its Python binding.  Importing it does not
touch the GPU; ``lib()`` loads the library and raises if it has not been built.
"""

from ._abi import NnpError  # noqa: F401
from ._abi import load as lib  # noqa: F401

__all__ = ["lib", "NnpError"]
