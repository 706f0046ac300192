"""CPU oracle (test infrastructure only; never imported by the product path)."""

from .seminaive import Fixpoint, sg, sg_batch, tc, tc_batch  # noqa: F401
from .triangles import triangles  # noqa: F401
from .keys import merge_runs, sort_keys  # noqa: F401
