"""cwcssa: bulk stochastic simulation of Calculus of Wrapped Compartments
models on AMD Instinct MI355X.

The work happens in the C-ABI library ``_lib/libcwcssa.so`` (HIP kernels
for gfx950); this package is its thin Python binding.
"""
from .abi import (CwcError, Context, Model, Run, Server, Stream, cwc_codegen, run_into,  # noqa: F401
                  cwc_model_describe, confidence, realign,
                  load,
                  LIB_PATH, SYMBOLS, MODE_PLAIN, MODE_PERSISTENT)
