"""lorax: a hierarchical sparse solver (extended sparsification with low-rank
compression of well-separated fill-in) for AMD MI355X (gfx950).

The compute path lives in the C-ABI library ``liblorax.so`` built from
``csrc/``; ``lorax`` is its thin ctypes binding.  ``workloads`` builds seeded
synthetic inputs.  Submodules are imported lazily so that importing the package
does not load the GPU library.
"""
__all__ = ["lorax", "workloads"]
