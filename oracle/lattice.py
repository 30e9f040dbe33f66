"""Oracle: periodic hypercubic lattices with colored edges (test infrastructure only).

The paper (Sec. 2.2.1, Model specification) defines the system on a graph of sites and
bonds, provides a ``Hypercube`` graph, and lets each bond carry an integer "color" that
selects the bond type. Here color 0 = nearest-neighbour (J1) bonds and color 1 =
next-nearest-neighbour diagonals (J2) of the square lattice.

Ordering convention (shared with the library only as a written convention, not code):
site s = sum_d x_d * L**d (x_0 fastest). Color-0 bonds are listed site by site, and for
each site dimension by dimension, as (s, s + e_d mod L). Color-1 bonds (2D only) are
listed site by site as (s, s + e_x + e_y), then (s, s + e_x - e_y).

Pinned by: the bond count and degree invariants (every site has degree 2d in color 0,
4 in color 1), and by the exact-diagonalisation energies of the Hamiltonians built on
these bonds (TFIM closed form, Bethe ansatz, 4x4 ED) in ``tests/test_oracle_exact.py``.
"""
import itertools

import numpy as np


def site_index(coords, L):
    """Row-major site index with the first coordinate fastest."""
    return int(sum(int(c) % L * L ** d for d, c in enumerate(coords)))


def hypercube(L, ndim, with_diagonals=False):
    """Return (bonds_by_color, sublattice) for an L**ndim periodic hypercube.

    bonds_by_color[c] is an int32 array [B_c, 2]; sublattice[s] = (sum of coordinates)
    mod 2, which is a proper two-coloring when L is even.
    """
    if L < 3:
        raise ValueError("periodic hypercube needs L >= 3 (L=2 would double bonds)")
    n = L ** ndim
    nn, nnn = [], []
    sub = np.zeros(n, dtype=np.int8)
    for s in range(n):
        coords = [(s // L ** d) % L for d in range(ndim)]
        sub[s] = sum(coords) % 2
        for d in range(ndim):
            c2 = list(coords)
            c2[d] += 1
            nn.append((s, site_index(c2, L)))
        if with_diagonals:
            if ndim != 2:
                raise ValueError("diagonal (J2) bonds are defined for the square lattice only")
            x, y = coords
            nnn.append((s, site_index((x + 1, y + 1), L)))
            nnn.append((s, site_index((x + 1, y - 1), L)))
    bonds = [np.array(nn, dtype=np.int32).reshape(-1, 2)]
    bonds.append(np.array(nnn, dtype=np.int32).reshape(-1, 2))
    return bonds, sub


def all_configs(n):
    """All 2**n spin configurations, sigma_i in {+1,-1}; row k has bit (n-1-i) of k set
    exactly when sigma_i = -1 (site 0 is the most significant bit, matching the order of
    Kronecker products with site 0 leftmost)."""
    out = np.empty((2 ** n, n), dtype=np.int8)
    for k, bits in enumerate(itertools.product((0, 1), repeat=n)):
        out[k] = 1 - 2 * np.array(bits, dtype=np.int8)
    return out
