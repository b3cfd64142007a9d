"""Seeded synthetic inputs (geometry, parameters, initial fields).

This package is shared by the GPU library's tests and benchmark and by the
FP64 reference; it contains no lattice Boltzmann arithmetic.
"""
from .case import (Case, MECH_PRE, MECH_POST, SCHEME_SNEW, SCHEME_SV, SCHEME_SPJ,
                   SCHEME_ABB)
from . import geometry, configs

__all__ = ["Case", "MECH_PRE", "MECH_POST", "SCHEME_SNEW", "SCHEME_SV", "SCHEME_SPJ",
           "SCHEME_ABB", "geometry", "configs"]
