"""Batched restarted PDHG for many LPs sharing one constraint matrix, on MI355X.

The solver is the HIP library ``libpdlpb.so`` (C ABI in include/pdlpb.h);
``paper_2601_21990_amd.pdlpb`` is its ctypes binding.
"""
import os as _os

LIB_PATH = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "libpdlpb.so")
