"""MI355X-native hot path of SMIwiz: staggered-grid acoustic FDTD modelling with CPML,
boundary-saving source-field reconstruction, adjoint propagation, FWI gradient and RTM image,
inside an evolving computing box.  The compute runs in hand-written HIP kernels (libsmi.so,
C ABI in include/smi.h); this package holds the ctypes binding, the autograd wrapper, the
shot server and the seeded synthetic inputs."""

__all__ = ["inputs", "binding", "autograd", "server", "build"]


def __getattr__(name):
    import importlib
    if name in __all__:
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
