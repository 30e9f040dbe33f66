"""Pins of the exact ground truth: closed forms and Bethe ansatz against sparse ED of
Hamiltonians assembled from Kronecker products of Pauli matrices."""
import os

import numpy as np
import pytest

from oracle import exact, lattice
from oracle.hamiltonian import HEISENBERG, TFIM, Model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "reference_energies.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            name, val, _ = line.split()
            out[name] = float(val)
    return out


@pytest.mark.parametrize("n,h", [(9, 1.3), (10, 1.0), (11, 0.7), (12, 1.5)])
def test_tfim_closed_form_matches_ed(n, h):
    bonds, sub = lattice.hypercube(n, 1)
    m = Model(n, 1, bonds, ham=TFIM, J=(1.0, 0.0), h=h)
    assert abs(exact.ground_energy(m)[0] - exact.tfim_ground_energy(n, 1.0, h)) < 1e-10


def test_tfim_closed_form_golden():
    assert abs(exact.tfim_ground_energy(10, 1.0, 1.0) - golden()["tfim_n10_h1"]) < 1e-13


def test_golden_lines_follow_from_the_oracle():
    # the computed lines of the golden file, re-derived (tests/golden/make_reference_energies.py)
    gd = golden()
    assert abs(exact.heisenberg_ring_bethe(20) - gd["heis_ring_n20"]) < 1e-12 * 36
    assert abs(exact.heisenberg_ring_bethe(40) - gd["heis_ring_n40"]) < 1e-12 * 71


@pytest.mark.parametrize("n", [20, 40, 80])
def test_bethe_ring_against_thermodynamic_limit(n):
    # Hulthen's infinite-chain energy 1 - 4 ln 2 per site (Pauli units) with the
    # conformal finite-size term -pi v c / (6 N^2) (v = 2 pi in Pauli units, c = 1); what
    # is left is the logarithmic correction, below 0.05 / N^2 at these sizes
    e = exact.heisenberg_ring_bethe(n) / n
    pred = 1.0 - 4.0 * np.log(2.0) - np.pi ** 2 / (3.0 * n * n)
    assert abs(e - pred) < 0.05 / (n * n), (e, pred)


@pytest.mark.parametrize("n", [10, 12, 16])
def test_bethe_matches_ed(n):
    bonds, sub = lattice.hypercube(n, 1)
    m = Model(n, 1, bonds, ham=HEISENBERG, J=(1.0, 0.0), sublattice=sub)
    e_ed = exact.ground_energy(m, sector_sz=0)[0]
    assert abs(e_ed - exact.heisenberg_ring_bethe(n)) < 1e-9 * abs(e_ed)


def test_marshall_rotation_keeps_spectrum():
    bonds, sub = lattice.hypercube(8, 1)
    m0 = Model(8, 1, bonds, ham=HEISENBERG, J=(1.0, 0.0), sublattice=sub)
    m1 = Model(8, 1, bonds, ham=HEISENBERG, J=(1.0, 0.0), sublattice=sub, marshall=True)
    e0 = np.linalg.eigvalsh(exact.dense_hamiltonian(m0))
    e1 = np.linalg.eigvalsh(exact.dense_hamiltonian(m1))
    assert np.allclose(e0, e1, atol=1e-12)
    # the rotated ground state has one sign (Marshall's theorem)
    w, v = np.linalg.eigh(exact.dense_hamiltonian(m1))
    g = v[:, 0]
    g = g[np.abs(g) > 1e-10]
    assert np.all(g.real > 0) or np.all(g.real < 0)


@pytest.mark.slow_ok
def test_4x4_heisenberg_and_j1j2_against_literature():
    gd = golden()
    bonds, sub = lattice.hypercube(4, 2, with_diagonals=True)
    m = Model(16, 1, bonds, ham=HEISENBERG, J=(1.0, 0.0), sublattice=sub)
    e = exact.ground_energy(m, sector_sz=0)[0]
    assert abs(e / 16 / 4 - gd["heis_4x4_per_site_spin_units"]) < 1e-6
    m2 = Model(16, 1, bonds, ham=HEISENBERG, J=(1.0, 0.5), sublattice=sub)
    e2 = exact.ground_energy(m2, sector_sz=0)[0]
    assert abs(e2 / 16 / 4 - gd["j1j2_4x4_j2_0.5_per_site_spin_units"]) < 1e-4
