"""Robust kernels on the squared Mahalanobis norm s = r^T Omega r
(test infrastructure, FP64).

Huber (Background, Eq. 7) is applied to s with threshold delta^2 (delta in
pixels, a reading: the paper names the kernel but not its parameterisation):

  rho(s) = s                        if s <= delta^2
  rho(s) = 2 delta sqrt(s) - delta^2  otherwise

rho and rho' are continuous at s = delta^2 (value delta^2, slope 1).  The
Gauss-Newton linearisation uses the IRLS weight w = rho'(s) only (no
second-order term), which keeps the normal matrix positive semi-definite.
"""
import numpy as np

SQUARED = 0
HUBER = 1


def rho(s, loss, delta):
    s = np.asarray(s, dtype=np.float64)
    if loss == SQUARED:
        return s.copy()
    d2 = delta * delta
    lin = 2.0 * delta * np.sqrt(np.maximum(s, d2)) - d2
    return np.where(s <= d2, s, lin)


def weight(s, loss, delta):
    """IRLS weight rho'(s)."""
    s = np.asarray(s, dtype=np.float64)
    if loss == SQUARED:
        return np.ones_like(s)
    d2 = delta * delta
    return np.where(s <= d2, 1.0, delta / np.sqrt(np.maximum(s, d2)))
