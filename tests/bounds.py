"""Element-wise error bound of an operator applied in BF16 storage.

Model (IEEE round to nearest, unit roundoff u = 2^-8 for BF16's 8 significant
bits): the input x and the links are rounded once on entry (|delta| <= u |v|
per complex entry, the real and imaginary parts rounded separately), products
and sums run in FP32 (their rounding, ~2^-24 per operation, is negligible
here), and the result is rounded once on output.  Each term D_ij x_j then
carries at most (2u + u^2) |D_ij| |x_j| and the output u |y_i|, so

    |y_i - (D x)_i| <= 2u (|D| |x|)_i + u |(D x)_i|   (+ FP32 terms).

The tests allow a factor 1.5 on each part for the FP32 terms and the spin
projection, which adds two rounded components before the link product.
"""
import numpy as np

U_BF16 = 2.0 ** -8


def bf16_bound_ratio(Y: np.ndarray, ref: np.ndarray, Dabs: np.ndarray, Xabs: np.ndarray) -> float:
    """max_i |Y_i - ref_i| / bound_i for rows of Y, ref (one right-hand side per row)."""
    bound = 3.0 * U_BF16 * (Dabs @ Xabs.T).T + 1.5 * U_BF16 * np.abs(ref)
    return float(np.max(np.abs(Y - ref) / bound))
