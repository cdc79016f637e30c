"""MI355X-native DDELM-NN: domain-decomposed extreme learning machines with a
coarse space and Neumann-Neumann acceleration, as HIP kernels behind a C ABI.

    from paper_2503_10032_amd import DDELMSolver, inputs
"""
from . import inputs  # noqa: F401

__all__ = ["DDELMSolver", "DDELMError", "inputs"]


def __getattr__(name):
    if name in ("DDELMSolver", "DDELMError"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
