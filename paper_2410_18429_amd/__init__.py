"""MI355X (gfx950) augmented-wavefield solver: batched CGLS for the
data-augmented Helmholtz systems of source-free wavefield reconstruction
inversion, the on-the-fly source-weight estimate, and the objective and its
gradient in the model.

The compute lives in libwri.so (HIP kernels + C ABI, include/wri.h); the
module `paper_2410_18429_amd.wri` is a ctypes binding over it.
"""
