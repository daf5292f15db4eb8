"""Seeded synthetic inputs for the random-walker solver.

This package only draws test volumes and seed maps. It holds none of the
solver's arithmetic (no weights, no Laplacian, no solve), so the CPU oracle
and the GPU path can both take their inputs from it without sharing method
code.
"""
from .volumes import (  # noqa: F401
    Case,
    sphere_case,
    blob_case,
    brickwise_blob_case,
    random_case,
    splitmix64,
    timeseries_case,
)
