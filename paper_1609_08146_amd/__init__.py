"""MI355X-native evaluation of the physical-optics Stratton-Chu integrals of a
field focused by a parabolic mirror (Dumont et al., arXiv:1609.08146).

The computation lives in the gfx950 shared library ``lib/libsc.so`` (C ABI in
``include/sc.h``); this package only marshals arguments.  Importing the
binding loads the library and fails loudly if it has not been built.
"""
from ._abi import (SC_FP32, SC_FP32_SPLIT, SC_FP64, ScError, load as load_library)  # noqa: F401
from .api import Context, Problem, Server, problem_from_workload, stencil_points  # noqa: F401

__all__ = ["Context", "Problem", "Server", "problem_from_workload", "stencil_points", "ScError", "SC_FP64",
           "SC_FP32_SPLIT", "SC_FP32", "load_library"]
