"""Cayley-graph growth on MI355X (gfx950).

Layer-by-layer breadth-first search from the identity of a permutation
group's Cayley graph: the layer sizes are the growth function (paper,
section "Reminder on Cayley graphs, diameters, growth"). The work runs in
hand-written HIP kernels behind the C ABI ``libcayleygrowth.so``
(``include/cayleygrowth.h``); this package is its thin Python binding.

The native library is loaded on first use, not at import, so that
``paper_2509_19162_amd.inputs`` can be imported without it.
"""

__all__ = ["growth", "growth_ex", "growth_batch", "GrowthQueue", "CGError"]


def __getattr__(name):
    if name in __all__:
        from . import api

        return getattr(api, name)
    raise AttributeError(name)
