"""MI355X-native decision engine for the out-of-bounds queries of a static
GPU bounds analysis: word-level normalisation + Tseitin CNF, cube splitting,
device unit propagation and bit-sliced exhaustive leaf evaluation on gfx950.

The C ABI (``include/scuba.h``) is the product; ``api`` is its Python
binding.  Importing the package loads nothing; ``api.Context`` loads
``libscuba.so`` and fails if it has not been built."""
from . import _lib  # noqa: F401

__all__ = ["api", "build"]
