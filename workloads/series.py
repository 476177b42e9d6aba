"""Truncated Taylor series, vectorised over many expansion points.

Used only to produce the caller-side inputs of the local part: curve and
density derivatives with respect to the tangent-line excursion xi at each
target's closest boundary point (Sec. 4, the local parametrization of the
curve and densities).  A series is stored as coefficients c[k] = g^(k)(0)/k!,
shape (K+1, n).
"""
import numpy as np

K = 4


class TS:
    __slots__ = ("c",)

    def __init__(self, c):
        self.c = np.asarray(c, dtype=np.float64)

    @staticmethod
    def const(v, n):
        c = np.zeros((K + 1, n))
        c[0] = v
        return TS(c)

    @staticmethod
    def var(n):
        c = np.zeros((K + 1, n))
        c[1] = 1.0
        return TS(c)

    def __add__(self, o):
        if isinstance(o, TS):
            return TS(self.c + o.c)
        c = self.c.copy()
        c[0] = c[0] + o
        return TS(c)

    __radd__ = __add__

    def __neg__(self):
        return TS(-self.c)

    def __sub__(self, o):
        return self + (-o)

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if not isinstance(o, TS):
            return TS(self.c * o)
        out = np.zeros_like(self.c)
        for i in range(K + 1):
            for j in range(K + 1 - i):
                out[i + j] += self.c[i] * o.c[j]
        return TS(out)

    __rmul__ = __mul__

    def recip(self):
        a = self.c
        b = np.zeros_like(a)
        b[0] = 1.0 / a[0]
        for k in range(1, K + 1):
            s = np.zeros_like(a[0])
            for j in range(1, k + 1):
                s += a[j] * b[k - j]
            b[k] = -s / a[0]
        return TS(b)

    def __truediv__(self, o):
        if isinstance(o, TS):
            return self * o.recip()
        return TS(self.c / o)

    def powers(self):
        """[1, g, g^2, ..., g^K] for a series with zero constant term."""
        n = self.c.shape[1]
        out = [TS.const(1.0, n)]
        for _ in range(K):
            out.append(out[-1] * self)
        return out

    def compose_into(self, outer):
        """outer(self) where outer is a coefficient array (K+1, n) and self(0)=0."""
        p = self.powers()
        acc = TS(np.zeros_like(self.c))
        for k in range(K + 1):
            acc = acc + p[k] * outer[k]
        return acc

    def integrate(self, c0):
        """Antiderivative with constant term c0 (truncated to order K)."""
        out = np.zeros_like(self.c)
        out[0] = c0
        for k in range(K):
            out[k + 1] = self.c[k] / (k + 1)
        return TS(out)

    def reversion(self):
        """Inverse series tau(xi) of xi(tau) = a1 tau + a2 tau^2 + ...; a1 != 0."""
        a1 = self.c[1]
        n = self.c.shape[1]
        x = TS.var(n)
        t = x / a1
        for _ in range(K):
            rest = TS(self.c.copy())
            rest.c[0] = 0.0
            rest.c[1] = 0.0
            t = (x - t.compose_series(rest)) / a1
        return t

    def compose_series(self, outer):
        """outer(self) where outer is a TS (its coefficients) and self(0)=0."""
        return self.compose_into(outer.c)

    def deriv(self, k):
        """k-th derivative at 0."""
        f = 1.0
        for i in range(2, k + 1):
            f *= i
        return self.c[k] * f


def sin_cos_shift(theta0, g):
    """(sin(theta0 + g), cos(theta0 + g)) for a series g with g(0) = 0."""
    p = g.powers()
    s = p[1] - p[3] * (1.0 / 6.0)
    c = p[0] - p[2] * 0.5 + p[4] * (1.0 / 24.0)
    s0, c0 = np.sin(theta0), np.cos(theta0)
    return s * c0 + c * s0, c * c0 - s * s0


def trig_shift_coeffs(freq, t0):
    """Taylor coefficients in tau of cos(freq*(t0+tau)) and sin(freq*(t0+tau))."""
    t0 = np.asarray(t0, dtype=np.float64)
    cs = np.zeros((K + 1, t0.size))
    sn = np.zeros((K + 1, t0.size))
    c0, s0 = np.cos(freq * t0), np.sin(freq * t0)
    fk = 1.0
    for k in range(K + 1):
        if k > 0:
            fk *= k
        w = freq ** k / fk
        # d^k/dtau^k cos(f(t0+tau)) = f^k cos(f t0 + k pi/2)
        m = k % 4
        dc = [c0, -s0, -c0, s0][m]
        ds = [s0, c0, -s0, -c0][m]
        cs[k] = w * dc
        sn[k] = w * ds
    return cs, sn
