"""MI355X (gfx950) implementation of RSAI(tol), the residual based sparse
approximate inverse of Jia & Kang (arXiv:1503.04500).

``rsai`` is the binding of the C ABI in ``include/rsai.h`` (librsai.so);
``gen`` builds seeded synthetic CSC inputs.
"""
