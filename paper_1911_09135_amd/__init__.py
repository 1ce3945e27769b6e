"""MI355X-native adaptive load balancer (ALB) for data-driven graph traversal.

The compute path is libalb.so (HIP for gfx950, C ABI in include/alb.h);
`paper_1911_09135_amd.alb` is its Python binding.  Importing the binding
fails loudly when the library is not built.
"""
__all__ = ["alb", "build"]
