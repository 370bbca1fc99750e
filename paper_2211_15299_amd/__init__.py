"""Homogeneous-support DFT on AMD MI355X (arXiv 2211.15299).

The transform runs in the HIP library built from csrc/ (libhidft.so, C ABI in
include/hidft.h); ``native`` is its ctypes binding.  Build with
``python -m paper_2211_15299_amd.build``.
"""
from .native import HiDFTError, Plan, analyze, lib  # noqa: F401

__all__ = ["HiDFTError", "Plan", "analyze", "lib"]
