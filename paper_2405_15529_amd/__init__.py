"""MI355X (gfx950) POD / tall-skinny SVD library after pyLOM (arXiv 2405.15529).

The compute path is the HIP library ``libpylom.so`` behind the C-ABI declared
in ``include/pylom.h``; ``api`` marshals PyTorch GPU tensors into it.
"""
from .api import (Context, PodResult, PylomError, context, matmul, pod, tree_plan, tsqr,  # noqa: F401
                  tsvd)
