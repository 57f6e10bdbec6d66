"""ecut: entanglement-cut bipartite H*psi on MI355X (gfx950).

The GPU library (libecut.so: host sector builder + HIP kernels behind the
C ABI in include/ecut.h) is loaded lazily by `paper_2605_07621_amd.ecut`;
importing the package itself loads nothing, so `paper_2605_07621_amd.inputs`
can be used without a GPU.
"""
__all__ = ["inputs", "ecut"]
