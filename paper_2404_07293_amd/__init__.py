"""MI355X-native coupled-wave-theory field synthesis (HIP library + binding).

The computation lives in libscw.so (include/scw.h); this package only loads it
and marshals arguments. Importing the package does not load the library;
``Context()`` does, and raises ImportError when it has not been built.
"""
from .scw import Context, Solution
from ._native import ScwError, LIB_PATH, load

__all__ = ["Context", "Solution", "ScwError", "LIB_PATH", "load"]
