"""Benelux-pair oracle: TEST INFRASTRUCTURE ONLY.

Plain CPU reference (trial-division radicals plus a hash-map join over the sets
{rad(x), rad(x+1)}) used by the tests, by the smoke check and by the benchmark's
CPU-baseline leg.  The product library never imports this package.  See
``benelux_oracle.cpp`` for the definitions it follows and the passages of the
paper they come from.
"""
from .oracle import (  # noqa: F401
    build,
    lib_path,
    rad,
    radicals,
    search,
    search_range,
    search_range_timed,
)
