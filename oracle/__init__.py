"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check of the build entry point and the CPU-baseline
leg of the benchmark may import this package.  The product path (the C-ABI
library under ``paper_2211_15299_amd`` and its Python binding) must never
import, call or link anything here; the two share no code.
"""
from .hidft_oracle import *  # noqa: F401,F403
from . import hidft_oracle  # noqa: F401
