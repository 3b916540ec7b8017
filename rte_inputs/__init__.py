"""Seeded synthetic inputs shared by the solver's tests, benchmark and the oracle.

This package only draws random numbers, lays out arrays and serialises
weights.  It contains none of the solver's arithmetic, so neither side of a
parity comparison can inherit a mistake from it.
"""
from . import configs, media, quadrature, weights  # noqa: F401
