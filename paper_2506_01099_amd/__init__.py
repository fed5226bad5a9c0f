"""MI355X-native (gfx950) search for Benelux pairs (arXiv:2506.01099).

The sieve of radicals and the exact hash-partitioned join run as HIP kernels in
libbenelux.so behind the C-ABI of include/benelux.h; this package is its thin
Python binding.
"""
from .api import BOTH, FIRST, SECOND, THIRD, VALUE_LIMIT, Benelux, Server, benelux_search, radical_segment  # noqa: F401
from ._lib import EXPORTS, LIB_PATH, BxError  # noqa: F401
