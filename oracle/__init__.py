"""CPU oracle package -- test infrastructure only.

Imported by the tests, the smoke check and the benchmark's CPU-baseline leg.
The GPU library and its Python binding never import it.
"""
from . import lbmz_oracle  # noqa: F401
