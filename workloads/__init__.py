"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds input generators only -- no step of the MINE method.  Both
the GPU library's tests and the FP64 oracle draw their inputs from here.
"""
from .gen import (  # noqa: F401
    sine_pair, relations_matrix, microarray_matrix, counts_matrix, uneven_stream,
    cpp_example, fig2_points, boundary_cases, RELATIONS,
)
