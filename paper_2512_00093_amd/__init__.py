"""RANMAR on MI355X (gfx950): seeding, exact jump-ahead and bulk generation.

A thin Python face of the C library ``libranmar.so`` (include/ranmar.h); every
function forwards to the C entry point of the same name.  Implements the
generator and jump-ahead of Haramoto & Suzuki, arXiv 2512.00093.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import RanmarError, lib  # noqa: F401
