"""radiotrace: FP64 eikonal ray tracing on MI355X.

GPU implementation of the method of RadioPropa (arXiv:1810.01780), section 2:
adaptive Cash-Karp integration of the ray equation through stratified or
gridded refractive-index fields, with planar boundaries that reflect the ray
and cast a refracted secondary carrying Fresnel amplitudes.

- ``binding``   : ctypes binding of the C ABI in include/radiotrace.h
- ``workloads`` : seeded synthetic scenes (media, boundaries, sources, rays)
- ``build``     : compiles the HIP library in-tree for gfx950
"""
__all__ = ["binding", "workloads", "build"]
