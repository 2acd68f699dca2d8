"""MI355X-native rendering path of CityGaussian (arXiv 2404.01133).

Block-wise level-of-detail selection (Sec. 3.3.2) feeding a differentiable
tile-based 3D Gaussian splatting rasterizer (Sec. 3.1, Eq. 1), as hand-written
HIP kernels for gfx950 behind the C ABI declared in include/gs.h.

Submodules are imported lazily so that the seeded generators (`synth`) can be
used without loading the HIP library.
"""
__all__ = ["synth", "gs", "render"]
