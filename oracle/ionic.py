"""Aliev-Panfilov ionic model (oracle; test infrastructure).

Sec. 5.1 of the paper gives the current and gating rate

    I(v, w) = k v (v - a)(v - 1) + v w
    R(v, w) = s (eps0 + mu1 w / (v + mu2)) (-w - k v (v - a - 1))

with g_a = g_s = k and the factor s = 1/4 printed in front of R.  Parameter
values are inputs (the synthetic workloads use k=8, a=0.15, eps0=0.002,
mu1=0.2, mu2=0.3, s=1/4); the paper's own values are a=0.1, eps1=0.01,
mu1=0.07, mu2=0.3.

Parameters are passed as a length-6 sequence (k, a, eps0, mu1, mu2, s).
"""
import numpy as np

K, A, EPS0, MU1, MU2, S = range(6)


def current(v, w, p):
    """I(v, w) = k v (v - a)(v - 1) + v w."""
    return p[K] * v * (v - p[A]) * (v - 1.0) + v * w


def rate(v, w, p):
    """R(v, w) = s (eps0 + mu1 w/(v + mu2)) (-w - k v (v - a - 1))."""
    return p[S] * (p[EPS0] + p[MU1] * w / (v + p[MU2])) * (-w - p[K] * v * (v - p[A] - 1.0))


def current_partials(v, w, p):
    """(dI/dv, dI/dw, dI/da)."""
    k, a = p[K], p[A]
    d_v = k * ((v - a) * (v - 1.0) + v * (v - 1.0) + v * (v - a)) + w
    d_w = v
    d_a = -k * v * (v - 1.0)
    return d_v, d_w, d_a


def rate_partials(v, w, p):
    """(dR/dv, dR/dw, dR/da) by the product rule on e(v,w) * g(v,w)."""
    k, a, eps0, mu1, mu2, s = (p[i] for i in range(6))
    e = eps0 + mu1 * w / (v + mu2)
    g = -w - k * v * (v - a - 1.0)
    e_v = -mu1 * w / (v + mu2) ** 2
    e_w = mu1 / (v + mu2)
    g_v = -k * (2.0 * v - a - 1.0)
    g_w = -1.0
    g_a = k * v
    return s * (e_v * g + e * g_v), s * (e_w * g + e * g_w), s * e * g_a


def as_params(p):
    return np.asarray(p, dtype=np.float64)
