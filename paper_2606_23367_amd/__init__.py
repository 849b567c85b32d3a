"""MI355X-native batched factor-model rebalancing solver.

The solver itself is the HIP library ``libfqp.so`` (kernels for gfx950 and a
C-ABI declared in ``include/fqp.h``); this package is its thin binding.
"""
from ._lib import STATUS_NAMES, SOLVED  # noqa: F401


def __getattr__(name):
    if name in ("Solver", "solve_batch", "to_device", "DeviceProblem",
                "pack_eligibility", "FqpFunction", "solve_differentiable", "subset"):
        from . import solver
        return getattr(solver, name)
    if name == "autotune":
        from .tune import autotune
        return autotune
    if name in ("audit_records", "queue_summary"):
        from . import audit
        return getattr(audit, name)
    raise AttributeError(name)
