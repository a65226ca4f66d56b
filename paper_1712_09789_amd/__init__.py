"""MI355X (gfx950) connected-components labelling: the block-based
coarse-to-fine method of Chen et al. (arXiv 1712.09789) as HIP kernels behind
a C ABI (include/ccl.h).

``paper_1712_09789_amd.ccl`` is the binding (``label``, ``label_batch``, ...);
``paper_1712_09789_amd.workloads`` draws seeded synthetic inputs.  The binding
is imported lazily so that the input generators work without the library.
"""

__all__ = ["ccl", "workloads", "label", "label_batch"]


def __getattr__(name):
    # import_module, not "from . import ccl": the latter asks this module for
    # the attribute first and would land here again
    import importlib
    if name in ("label", "label_batch", "label_local"):
        return getattr(importlib.import_module(__name__ + ".ccl"), name)
    if name == "ccl":
        return importlib.import_module(__name__ + ".ccl")
    raise AttributeError(name)
