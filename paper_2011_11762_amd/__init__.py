"""Block-sparse quadtree matrix multiply for AMD MI355X (gfx950).

The compute path lives in a HIP shared library with a C ABI (``include/qbsm.h``);
``paper_2011_11762_amd.qbsm`` is its thin Python binding.  Importing the
package itself loads nothing, so the seeded workload generators in
``paper_2011_11762_amd.workloads`` can be used without a GPU.
"""
import importlib

__all__ = ["qbsm", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
