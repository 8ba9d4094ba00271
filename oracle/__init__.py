"""The oracle: plain CPU complex128 implementation of CBC and the tensor-network metrics.

TEST INFRASTRUCTURE ONLY -- imported by tests, the smoke check and the benchmark's CPU-baseline leg,
never by the library. Shares no code with the GPU path.
"""
from .cbc import cbc_tt, cbc_tree, truncate_joined, lq  # noqa: F401
from . import tn  # noqa: F401
from .src import src_tree  # noqa: F401
from .dm import dm_tree  # noqa: F401
from .zipup import zipup_tree  # noqa: F401
