"""Multifrontal log-det barrier kernels for AMD MI355X (gfx950).

The HIP library ``libmfb.so`` (C ABI in ``include/mfb.h``) evaluates the
barrier f(X) = -log det X on a filled sparsity pattern, its gradient
(projected inverse), Hessian products and their inverse, and the completion
recursion of the dual barrier.  ``paper_1203_2742_amd.mfb`` is the Python
binding.
"""
__all__ = ["mfb"]
