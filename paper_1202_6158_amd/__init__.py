"""D-iteration PageRank on AMD MI355X (gfx950).

The solver is libdi.so (HIP kernels behind the C ABI in include/di.h); the
Python side is the ctypes binding in :mod:`paper_1202_6158_amd.di`, imported
lazily so that building does not require the library to exist yet.
"""
import os

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libdi.so")


def build(verbose: bool = False) -> str:
    from . import compile_lib as _b
    return _b.build(verbose=verbose)


def load():
    """Import the binding (raises ImportError if libdi.so is missing)."""
    from . import di
    return di
