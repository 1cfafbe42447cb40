"""Independent brute-force evaluators used to pin the oracle on tiny inputs.

The cardinal B-spline here comes from the truncated-power formula (the
(n+1)-fold convolution of the unit box), not from the piecewise polynomials
the oracle uses, and the transfers visit every grid node instead of a kernel
support, so a wrong support, base node or spline piece in the oracle shows up
as a mismatch.
"""
import math

import numpy as np


def bspline_tp(n: int, t: float) -> float:
    """Centred cardinal B-spline of degree n at t via truncated powers:
    (1/n!) sum_k (-1)^k C(n+1,k) (t + (n+1)/2 - k)_+^n."""
    s = 0.0
    for k in range(n + 2):
        u = t + (n + 1) / 2.0 - k
        if u > 0:
            s += (-1) ** k * math.comb(n + 1, k) * u ** n
    return s / math.factorial(n)


def bspline_tp_deriv(n: int, t: float) -> float:
    s = 0.0
    for k in range(n + 2):
        u = t + (n + 1) / 2.0 - k
        if u > 0:
            s += (-1) ** k * math.comb(n + 1, k) * n * u ** (n - 1)
    return s / math.factorial(n)


def node_grid(cells, dx):
    axes = [np.arange(c + 1) for c in cells]
    mesh = np.meshgrid(*axes, indexing="ij")
    idx = np.stack([m.reshape(-1) for m in mesh], axis=1)
    return idx, idx * dx


def weight_all_nodes(degree, cells, dx, xp):
    """w_ip and grad w_ip at every node (brute force), in meshgrid 'ij' order."""
    idx, xi = node_grid(cells, dx)
    d = len(cells)
    w = np.ones(len(idx))
    one = np.zeros((len(idx), d))
    dw = np.zeros((len(idx), d))
    for j in range(len(idx)):
        t = [(xp[a] - xi[j, a]) / dx for a in range(d)]
        n_a = [bspline_tp(degree, ta) for ta in t]
        dn_a = [bspline_tp_deriv(degree, ta) / dx for ta in t]
        w[j] = np.prod(n_a)
        for a in range(d):
            g = dn_a[a]
            for b in range(d):
                if b != a:
                    g *= n_a[b]
            dw[j, a] = g
    return idx, xi, w, dw


def p2g_all_nodes(degree, cells, dx, x, v, B, m):
    """m_i and (m v)_i of Sec. 3.2 summed over every (particle, node) pair,
    with D_p formed over every node too.  Returns arrays in 'ij' order."""
    d = len(cells)
    idx, xi, _, _ = weight_all_nodes(degree, cells, dx, x[0])
    gm = np.zeros(len(idx))
    gmv = np.zeros((len(idx), d))
    for p in range(len(m)):
        _, _, w, _ = weight_all_nodes(degree, cells, dx, x[p])
        r = xi - x[p]
        D = np.einsum("j,ja,jb->ab", w, r, r)
        C = B[p] @ np.linalg.inv(D)
        gm += w * m[p]
        gmv += (w * m[p])[:, None] * (v[p][None, :] + r @ C.T)
    return idx, gm, gmv


def ij_to_oracle(idx, cells):
    """Map 'ij' ordered node indices to the oracle's linear node index
    ix + N0*(iy + N1*iz)."""
    nodes = [c + 1 for c in cells]
    lin = np.zeros(len(idx), dtype=np.int64)
    for a in reversed(range(len(cells))):
        lin = lin * nodes[a] + idx[:, a]
    return lin
