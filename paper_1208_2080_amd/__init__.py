"""swmi: Swendsen-Wang multi-cluster sweeps of the 2D q-state Potts model on one
AMD Instinct MI355X, as hand-written HIP kernels behind a C ABI (include/sw.h).

``Lattice`` / ``Batch`` and friends live in ``binding`` and are imported lazily
(they need torch); ``workloads`` holds the seeded synthetic inputs.
"""
__all__ = ["Lattice", "Batch", "Group", "SwError", "threshold", "workspace_bytes", "tile_count", "derived", "lib"]


def __getattr__(name):
    if name in __all__:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
