"""Runs CPU test files in this process against the sanitizer builds of the
host code: the oracle (ORC_LIB) and the library's host-only sources
(PP_HOST_SAN_LIB: region polygons and the drift map).  Started by
test_sanitizers.py with the sanitizer runtime preloaded."""
import ctypes
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2411_01919_amd import _native as N  # noqa: E402

assert hasattr(ctypes.CDLL(None), "__asan_init"), "the AddressSanitizer runtime is not loaded"
SAN = ctypes.CDLL(os.environ["PP_HOST_SAN_LIB"])
assert hasattr(SAN, "pp_region_polygons") and hasattr(SAN, "pp_map_integrate")
REAL = N.lib()  # the regular build, for the entry points the sanitizer build does not hold


class _Both:
    """Each entry point from the sanitizer build when it holds it, else from the regular build."""

    def __getattr__(self, name):
        fn = getattr(SAN, name, None)
        if fn is None:
            return getattr(REAL, name)
        res, args = N.SIGNATURES[name]
        fn.restype = res
        fn.argtypes = args
        return fn


N._lib = _Both()

sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", "-m", "not gpu", *sys.argv[1:]]))
