"""Plain FP64 CPU oracle for HOSCF / iHOSCF (best rank-one approximation of
dense higher-order tensors, arXiv 2403.01778).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything in
this package.  The product path (the HIP library and its Python binding) never
imports it, and it imports nothing from the product: the two share no kernels,
headers, helpers, tables or pre/post-processing.

Every function is written from the paper's definitions, in its order and
notation, with a NumPy/LAPACK primitive (tensordot, eigh, solve, svd) as the
only library steps.  Pins against values the paper and the mathematics fix
live in ``tests/test_oracle_*.py``.
"""
from .hoscf_oracle import *  # noqa: F401,F403
from . import quant  # noqa: F401
