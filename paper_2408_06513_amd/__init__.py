"""MI355X (gfx950) scatterplot regularisation with integral images.

Rave, Molchanov and Linsen, "De-cluttering Scatterplots with Integral Images"
(arXiv 2408.06513): splat + smooth the sample density, compute the axis and
45-degree tilted integral images, derive the per-texel density-equalising
deformation and move every sample by bilinear interpolation, iterated.

``capi`` is the binding of the C ABI (include/inim.h, libinim.so);
``datagen`` draws the seeded synthetic inputs.  Importing the package does not
load the HIP library; the first call does, and fails loudly if it is missing.
"""
__all__ = ["capi", "datagen", "build"]
