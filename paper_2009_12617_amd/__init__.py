"""MI355X-native smooth particle-mesh Ewald (SPME) reciprocal-space step.

    from paper_2009_12617_amd import Plan
    plan = Plan(K=64, order=4, beta=0.34, max_atoms=65535)
    forces, ev = plan.step(pos, q, box)      # device float64 tensors

The HIP library (libspme.so, C ABI in include/spme.h) does all the work;
PyTorch only provides device memory and streams.  Submodules are imported
lazily so that `paper_2009_12617_amd.inputs` works without torch or a GPU.
"""

__all__ = ["Plan", "Batch", "BatchPool", "KERNEL_NAMES", "RealSpace"]


def __getattr__(name):
    if name in ("Plan", "Batch", "BatchPool", "KERNEL_NAMES", "TUNE_CANDIDATES"):
        from . import plan as _plan
        return getattr(_plan, name)
    if name == "RealSpace":
        from . import realspace as _rs
        return _rs.RealSpace
    raise AttributeError(name)
