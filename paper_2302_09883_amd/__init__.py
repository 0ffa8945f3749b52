"""DWT-compressed stencil simulation on AMD Instinct MI355X (gfx950).

The compute path is the HIP library ``liblbmz.so`` built from ``csrc/``; this
package only exposes its C ABI (``include/lbmz.h``) to Python.
"""
from .lbmz import (  # noqa: F401
    Context,
    LbmzError,
    Net,
    library,
    LIB_PATH,
)
