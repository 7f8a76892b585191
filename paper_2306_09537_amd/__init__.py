"""MI355X-native batched quadrotor-swarm stepper (QuadSwarm, arXiv 2306.09537).

``QuadSwarm`` wraps the C ABI of ``libquadswarm.so`` (HIP kernels for
gfx950); ``workloads`` draws seeded synthetic inputs.  Importing the package
does not load the library; the first call that needs it does, and raises if
it is missing.
"""
from . import workloads  # noqa: F401


def __getattr__(name):
    if name in ("QuadSwarm", "QuadSwarmError", "lib"):
        from . import quadswarm
        return getattr(quadswarm, name)
    raise AttributeError(name)
