"""Seeded synthetic inputs (farm networks, model definitions, small test systems).

Inputs only: this package computes no step of the simulation method. It is the
one module that both the oracle's tests and the GPU path read from.
"""
from .problem import ENTER, EXIT, EXTERNAL, INTERNAL, KIND_NAMES, Problem  # noqa: F401
from . import synth  # noqa: F401
