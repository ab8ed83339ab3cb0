"""MI355X (gfx950) Lennard-Jones Verlet-list library: cell binning, neighbor
list build and LJ forces / energy / virial as hand-written HIP kernels behind
the C ABI of include/lj.h.

Importing the package touches neither the GPU nor the compiled library; the
binding `paper_1806_05713_amd.lj` loads liblj.so on first use.
"""
__all__ = ["lj", "synth", "build"]
