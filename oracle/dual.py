"""Vectorised forward-mode dual numbers (test infrastructure, FP64).

A Dual holds a value array v of shape (N,) and a derivative array d of shape
(N, K): K partial derivatives per element.  The paper (Sec. IV-C) computes
Jacobian columns by seeding one infinitesimal component per input; here all K
components are carried at once, vectorised over N residual evaluations.  This
is a derivative route independent of the closed-form Jacobians of the GPU
kernels.
"""
import numpy as np


class Dual:
    __slots__ = ("v", "d")

    def __init__(self, v, d):
        self.v = np.asarray(v, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)

    # --- helpers -----------------------------------------------------------
    @staticmethod
    def _split(o):
        if isinstance(o, Dual):
            return o.v, o.d
        return np.asarray(o, dtype=np.float64), None

    # --- arithmetic --------------------------------------------------------
    def __add__(self, o):
        ov, od = Dual._split(o)
        return Dual(self.v + ov, self.d if od is None else self.d + od)

    __radd__ = __add__

    def __sub__(self, o):
        ov, od = Dual._split(o)
        return Dual(self.v - ov, self.d if od is None else self.d - od)

    def __rsub__(self, o):
        ov, od = Dual._split(o)
        return Dual(ov - self.v, -self.d if od is None else od - self.d)

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __mul__(self, o):
        ov, od = Dual._split(o)
        d = self.d * ov[..., None]
        if od is not None:
            d = d + od * self.v[..., None]
        return Dual(self.v * ov, d)

    __rmul__ = __mul__

    def __truediv__(self, o):
        ov, od = Dual._split(o)
        q = self.v / ov
        d = self.d / ov[..., None]
        if od is not None:
            d = d - od * (q / ov)[..., None]
        return Dual(q, d)

    def __rtruediv__(self, o):
        ov, od = Dual._split(o)
        q = ov / self.v
        d = -self.d * (q / self.v)[..., None]
        if od is not None:
            d = d + od / self.v[..., None]
        return Dual(q, d)


def value(x):
    return x.v if isinstance(x, Dual) else np.asarray(x, dtype=np.float64)


def sqrt(x):
    if not isinstance(x, Dual):
        return np.sqrt(x)
    s = np.sqrt(x.v)
    return Dual(s, x.d * (0.5 / s)[..., None])


def sin(x):
    if not isinstance(x, Dual):
        return np.sin(x)
    return Dual(np.sin(x.v), x.d * np.cos(x.v)[..., None])


def cos(x):
    if not isinstance(x, Dual):
        return np.cos(x)
    return Dual(np.cos(x.v), x.d * (-np.sin(x.v))[..., None])


def where(cond, a, b):
    """Elementwise select between two Duals (or plain arrays)."""
    if not isinstance(a, Dual) and not isinstance(b, Dual):
        return np.where(cond, a, b)
    av, ad = Dual._split(a)
    bv, bd = Dual._split(b)
    n = av.shape[0] if av.ndim else bv.shape[0]
    k = (ad if ad is not None else bd).shape[-1]
    if ad is None:
        ad = np.zeros((n, k))
    if bd is None:
        bd = np.zeros((n, k))
    return Dual(np.where(cond, av, bv), np.where(cond[..., None], ad, bd))


def seed(values):
    """Turn an (N, K) array of inputs into K Duals whose derivative is the
    K x K identity for every element (one infinitesimal per input)."""
    values = np.asarray(values, dtype=np.float64)
    n, k = values.shape
    out = []
    for c in range(k):
        d = np.zeros((n, k))
        d[:, c] = 1.0
        out.append(Dual(values[:, c].copy(), d))
    return out
