"""One classical Gram-Schmidt pass of the Lanczos full reorthogonalisation.

Test infrastructure only (see the package docstring).

Sec. 4.2 (Eqs. Lanczos, LanczosAlphaBeta and the full reorthogonalisation
that keeps the Lanczos vectors M-orthonormal): a new vector x is made
M-orthogonal to the columns of B = [v_1 ... v_m] by subtracting its
M-projection.  With W = M B precomputed, the M-inner products are plain
inner products with W:

    c = W^T x,        x_new = x - B c.

Written out here from that definition with a matrix-vector product of the
full matrices; no blocking or reordering.
"""
import numpy as np


def cgs_pass(W, B, x):
    """c = W^T x and x - B c for column blocks W, B (n x m) and x (n).

    Returns (c, x_new); the inputs are not modified."""
    W = np.asarray(W, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    c = W.T @ x
    return c, x - B @ c
