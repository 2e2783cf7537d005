"""cwcssa: bulk stochastic simulation of Calculus of Wrapped Compartments
models on AMD Instinct MI355X.

The work happens in the C-ABI library ``_lib/libcwcssa.so`` (HIP kernels
for gfx950); this package is its thin Python binding.
"""
from .abi import (CwcError, Context, GModel, Model, Run, Server, Stream, cwc_codegen,  # noqa: F401
                  gcodegen, run_into,
                  cwc_model_describe, confidence, realign,
                  load,
                  LIB_PATH, SYMBOLS, MODE_PLAIN, MODE_PERSISTENT)
