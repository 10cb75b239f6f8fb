"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only draws random inputs: star-shaped polygons snapped to the
2^-30 coordinate lattice, the square data space that holds them, and random
sorted interval lists for join tests. It holds none of the filter's
arithmetic (no rasterisation, no Hilbert ordering, no joins), so the oracle
and the GPU library can both consume its output without sharing method code.
"""

from .polygons import (  # noqa: F401
    LATTICE,
    PolygonSet,
    star_polygons,
    snap,
)
from .grid import Grid, grid_covering  # noqa: F401
from .intervals import random_lists, complement_list, sub_lists, ListSet  # noqa: F401
from . import configs  # noqa: F401
from . import partitions  # noqa: F401
from . import linestrings  # noqa: F401
