"""Hyper-dual numbers for exact first and second directional derivatives.

A hyper-dual number  x = a + b e1 + c e2 + d e1e2  with e1^2 = e2^2 = 0 carries
the value a, the derivatives b (direction 1) and c (direction 2) and the mixed
second derivative d.  Evaluating R1_h on  w + e1 sigma + e2 dw  therefore gives

    a = R1(w),  b = R1'(w) sigma = R2(w, sigma),  c = R1'(w) dw,
    d = R1''(w)[sigma, dw] = (d R2 / d w) dw,

which is how the oracle defines R2 (Eq. DGSEM_wtt is the directional
derivative of Eq. DGSEM_wt along sigma) and the Hessian contribution of the
extended Jacobian (Eq. nonlinear_eqsys).  Components are NumPy arrays (real
or complex, so complex-step checks can run through the same code).

Non-smooth functions follow fixed tie rules: |x| takes the branch of
sign(Re a) with sign(0) = +1; max(x, y) takes x when Re a_x >= Re a_y.
"""
import numpy as np


class HD:
    __slots__ = ("a", "b", "c", "d")
    __array_ufunc__ = None          # make ndarray (op) HD defer to HD's reflected operators

    def __init__(self, a, b=None, c=None, d=None):
        self.a = a
        z = None
        if b is None or c is None or d is None:
            z = np.zeros_like(a)
        self.b = z if b is None else b
        self.c = z if c is None else c
        self.d = z if d is None else d

    # ---- arithmetic -------------------------------------------------------
    def __add__(self, o):
        if isinstance(o, HD):
            return HD(self.a + o.a, self.b + o.b, self.c + o.c, self.d + o.d)
        return HD(self.a + o, self.b, self.c, self.d)

    __radd__ = __add__

    def __neg__(self):
        return HD(-self.a, -self.b, -self.c, -self.d)

    def __sub__(self, o):
        if isinstance(o, HD):
            return HD(self.a - o.a, self.b - o.b, self.c - o.c, self.d - o.d)
        return HD(self.a - o, self.b, self.c, self.d)

    def __rsub__(self, o):
        return HD(o - self.a, -self.b, -self.c, -self.d)

    def __mul__(self, o):
        if isinstance(o, HD):
            return HD(self.a * o.a,
                      self.a * o.b + self.b * o.a,
                      self.a * o.c + self.c * o.a,
                      self.a * o.d + self.b * o.c + self.c * o.b + self.d * o.a)
        return HD(self.a * o, self.b * o, self.c * o, self.d * o)

    __rmul__ = __mul__

    def _apply(self, f0, f1, f2):
        """g(x) for a scalar function with value f0, first f1 and second f2 derivative at a."""
        return HD(f0, f1 * self.b, f1 * self.c, f1 * self.d + f2 * self.b * self.c)

    def reciprocal(self):
        inv = 1.0 / self.a
        return self._apply(inv, -inv * inv, 2.0 * inv * inv * inv)

    def __truediv__(self, o):
        if isinstance(o, HD):
            return self * o.reciprocal()
        return HD(self.a / o, self.b / o, self.c / o, self.d / o)

    def __rtruediv__(self, o):
        return self.reciprocal() * o


def sqrt(x):
    if isinstance(x, HD):
        s = np.sqrt(x.a)
        return x._apply(s, 0.5 / s, -0.25 / (s * x.a))
    return np.sqrt(x)


def _re(v):
    return np.real(v)


def absval(x):
    """|x| with sign(0) = +1; complex-step safe (branch on the real part)."""
    a = x.a if isinstance(x, HD) else x
    sgn = np.where(_re(a) >= 0.0, 1.0, -1.0)
    return x * sgn


def maxval(x, y):
    """max(x, y), choosing x on ties; branch on the real part."""
    ax = x.a if isinstance(x, HD) else x
    ay = y.a if isinstance(y, HD) else y
    pick = _re(ax) >= _re(ay)
    if isinstance(x, HD) or isinstance(y, HD):
        x = x if isinstance(x, HD) else HD(x)
        y = y if isinstance(y, HD) else HD(y)
        return HD(np.where(pick, x.a, y.a), np.where(pick, x.b, y.b),
                  np.where(pick, x.c, y.c), np.where(pick, x.d, y.d))
    return np.where(pick, x, y)


def value(x):
    return x.a if isinstance(x, HD) else x


def part(x, which):
    """Extract component 'a', 'b', 'c' or 'd' (plain arrays count as value only)."""
    if isinstance(x, HD):
        return getattr(x, which)
    return x if which == "a" else np.zeros_like(x)
