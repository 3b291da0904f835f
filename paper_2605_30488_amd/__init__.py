"""ds3: dense Sim(3) back-end of collaborative monocular dense SLAM (CoMo3R-SLAM, Sec. III) for AMD
MI355X. Bidirectional projective pointmap matching, gauge synchronisation and Gauss-Newton refinement
of the unified Sim(3) keyframe graph, as hand-written HIP kernels behind the C ABI in include/ds3.h.

The binding loads libds3.so lazily and raises when it is missing; nothing here computes on the CPU."""
from ._lib import DS3Error, exported_names, load  # noqa: F401

__all__ = ["DS3Error", "exported_names", "load", "api"]


def __getattr__(name):
    if name == "api":
        import importlib
        return importlib.import_module(__name__ + ".api")
    raise AttributeError(name)
