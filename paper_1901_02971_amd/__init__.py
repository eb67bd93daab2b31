"""MI355X sparsified nested dissection (spaND) solver.

The compute path lives in the HIP library ``libspand.so`` (C ABI in
``include/spand.h``); ``paper_1901_02971_amd.spand`` is a thin ctypes binding.
"""
from .spand import (SPAND_BF16X3, SPAND_FP32, SPAND_FP64, Solver, SpandError,  # noqa: F401
                    exported_symbols, factor_batch, library_path, load_library, solve_batch)
