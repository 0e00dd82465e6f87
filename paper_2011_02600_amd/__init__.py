"""MI355X (gfx950) upwind summation-by-parts solver for 3D elastic waves on a
boundary-conforming curvilinear block (Duru, Fung & Williams,
arXiv:2011.02600).

The numerical work runs in the HIP library libsbp.so (C ABI: include/sbp.h);
``paper_2011_02600_amd.sbp`` is its ctypes binding.
"""
__all__ = ["sbp"]
