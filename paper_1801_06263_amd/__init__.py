"""MI355X (gfx950) one-step spectral-CT reconstruction by MOCCA with
block-diagonal step preconditioning (arXiv 1801.06263).

The compute path is the HIP library libosscir.so (C ABI in include/osscir.h);
``paper_1801_06263_amd.osscir`` is its thin binding.
"""
from .osscir import Batch, Params, Plan, State, load_library, version  # noqa: F401
