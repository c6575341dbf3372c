"""Oracle values of single sites of a large lattice, from small windows.

One time step of the Chebyshev scheme (Sect. 2.2) applies a polynomial of
degree M in H~, so psi after K steps at site i depends only on psi_0 and the
on-site terms within graph distance K*M of i; so does a polynomial of H~
restricted to any sub-lattice that contains that ball.  On the brick-wall
ribbon (eq. (model)) and the 1D chain each bond changes one grid coordinate
by one, so the ball lies inside the grid window of half-width K*M (in both
coordinates) around i.  The oracle propagates that window with the full
lattice's plan (the same a, b and weights) and gives psi_K at i up to
rounding order, for lattices far too large to propagate whole on the CPU.

The brick wall's bond pattern depends on the parity of x + y: windows start
at an even x0 + y0 so the sub-lattice has the same bonds.
"""
from __future__ import annotations

import numpy as np

import oracle as O


def _ribbon_window(width, length, y, x, R):
    y0, y1 = max(0, y - R), min(width, y + R + 1)
    x0, x1 = max(0, x - R), min(length, x + R + 1)
    if (x0 + y0) % 2:  # keep the brick wall's parity: widen by one
        if x0 > 0:
            x0 -= 1
        else:
            y0 -= 1
    return y0, y1, x0, x1


def ribbon_sites(width, length, edge, eps, psi0, plan, K, sites):
    """psi_K at the given (y, x) sites of a width x length ribbon, each from
    the oracle on a window around it (see module docstring)."""
    R = K * plan.M + 1
    eps2 = np.asarray(eps).reshape(width, length)
    psi2 = np.asarray(psi0).reshape(width, length)
    out = np.zeros(len(sites), dtype=np.complex128)
    for j, (y, x) in enumerate(sites):
        y0, y1, x0, x1 = _ribbon_window(width, length, int(y), int(x), R)
        w, l = y1 - y0, x1 - x0
        H = O.honeycomb(w, l, np.ascontiguousarray(eps2[y0:y1, x0:x1]).reshape(-1), edge=edge)
        p = O.propagate(H, plan, np.ascontiguousarray(psi2[y0:y1, x0:x1]).reshape(-1), K)
        out[j] = p[(y - y0) * l + (x - x0)]
    return out


def chain_sites(V, dx, psi0, plan, K, sites):
    """psi_K at the given sites of a 1D chain (Sect. 3.1 Hamiltonian), each
    from the oracle on the window of half-width K*M + 1 around it."""
    R = K * plan.M + 1
    n = len(V)
    out = np.zeros(len(sites), dtype=np.complex128)
    for j, i in enumerate(sites):
        a, b = max(0, int(i) - R), min(n, int(i) + R + 1)
        H = O.chain1d(np.ascontiguousarray(V[a:b]), dx)
        p = O.propagate(H, plan, np.ascontiguousarray(psi0[a:b]), K)
        out[j] = p[int(i) - a]
    return out


def ribbon_sample_sites(width, length, count, seed, strips=(54, 56, 58, 60, 62)):
    """Sites to sample on a ribbon: the four corners, both edges' ends, the
    last rows and columns (the partial strip and chunk at the far borders),
    both sides of strip boundaries for the strip widths of the multi-order
    walks (66 - 2D columns for D orders per pass), and `count` seeded sites."""
    from workloads import uniform01
    pts = {(0, 0), (0, length - 1), (width - 1, 0), (width - 1, length - 1),
           (width // 2, length - 1), (width // 2, 0), (0, length // 2), (width - 1, length // 2),
           (width - 2, length - 2), (1, length - 3)}
    u = uniform01(seed ^ 0x51D, 2 * len(strips))
    for j, s in enumerate(strips):
        k = 1 + int(u[2 * j] * max(1, length // s - 1))
        y = int(u[2 * j + 1] * width)
        for x in (k * s - 1, k * s):
            if 0 <= x < length:
                pts.add((y, x))
        last = (length - 1) // s * s  # first column of the last, partial strip
        pts.add((width - 1 - y, last))
        if last > 0:
            pts.add((width - 1 - y, last - 1))
    u = uniform01(seed, 2 * count)
    for k in range(count):
        pts.add((int(u[2 * k] * width), int(u[2 * k + 1] * length)))
    return sorted(pts)
