"""MI355X (gfx950) k-point ISDF: fit, Coulomb kernel and fragment ERIs.

The compute path is the HIP library ``libisdf_gfx950.so`` behind the C ABI of
``include/isdf.h``; :mod:`paper_2601_16379_amd.isdf` is its ctypes binding.
"""
from .isdf import (Isdf, IsdfError, load_library, isdf_plan_bytes,  # noqa: F401
                   isdf_storage_model_bytes, isdf_version, select_points, EXPORTS, LIB_PATH)
