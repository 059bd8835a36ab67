"""MI355X (gfx950) Shepard IDW: all-pairs sweep, adjoint and batched form behind the C ABI
of libidw.so (include/idw.h).

Submodules: ``api`` (point descriptors, forward/backward, autograd Function, LOO fit),
``batched`` (many instances in one graph launch), ``workloads`` (seeded synthetic inputs),
``build`` (hipcc build of libidw.so).  Importing the package itself loads nothing.
"""

__all__ = ["api", "workloads", "build"]


def __getattr__(name):
    if name in ("api", "workloads", "build", "batched"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
