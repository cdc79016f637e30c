"""MI355X-native DDELM-NN: domain-decomposed extreme learning machines with a
coarse space and Neumann-Neumann acceleration, as HIP kernels behind a C ABI.

    from paper_2503_10032_amd import DDELMSolver, inputs
"""
from . import inputs  # noqa: F401

__all__ = ["DDELMSolver", "DDELMError", "inputs", "release_cached_memory"]


def release_cached_memory() -> None:
    """Hand the device memory, events, streams and pinned buffers that the
    library keeps from destroyed solvers back to the runtime."""
    from . import _lib
    st = _lib.load().ddelm_release_cached_memory()
    if st != 0:
        raise RuntimeError(f"ddelm_release_cached_memory failed ({_lib.STATUS_NAMES.get(st, st)})")


def __getattr__(name):
    if name in ("DDELMSolver", "DDELMError"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
