"""MI355X-native sparse-block reaction-diffusion (Stark & Sbalzarini, arXiv 2304.11165).

The compute path is librd.so (HIP for gfx950 + host C++), declared in
include/rd.h.  ``paper_2304_11165_amd.rd`` is its thin ctypes binding; it is
imported on first use so that ``paper_2304_11165_amd.build`` runs without a
built library.
"""

FACE = {"-x": 0, "+x": 1, "-y": 2, "+y": 3, "-z": 4, "+z": 5}

_EXPORTS = ("Batch", "Geometry", "RDError", "Sim")


def __getattr__(name):
    if name in _EXPORTS:
        from . import rd

        return getattr(rd, name)
    raise AttributeError(name)
