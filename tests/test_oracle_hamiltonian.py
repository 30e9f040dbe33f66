"""Pins of the oracle local energy (Eq. 5) against H assembled from Pauli Kronecker
products: row identity E_loc(sigma) = (H psi)(sigma) / psi(sigma), the full-sum identity
<E_loc>_{|psi|^2} = <psi|H|psi>/<psi|psi>, and special cases."""
import numpy as np
import pytest

import synth
from oracle import exact, hamiltonian, lattice, rbm
from oracle.hamiltonian import HEISENBERG, TFIM, Model


def models():
    b1, s1 = lattice.hypercube(8, 1)
    b2, s2 = lattice.hypercube(4, 2, with_diagonals=True)
    b3, s3 = lattice.hypercube(3, 2, with_diagonals=True)
    return {
        "tfim8": Model(8, 8, b1, ham=TFIM, J=(1.0, 0.0), h=0.8, sublattice=s1),
        "heis8": Model(8, 16, b1, ham=HEISENBERG, J=(1.0, 0.0), sublattice=s1, move=1),
        "heis8_marshall": Model(8, 16, b1, ham=HEISENBERG, J=(1.0, 0.0), sublattice=s1, marshall=True, move=1),
        "j1j2_4x4_marshall": Model(16, 16, b2, ham=HEISENBERG, J=(1.0, 0.5), sublattice=s2, marshall=True, move=1),
        "j1j2_3x3": Model(9, 9, b3, ham=HEISENBERG, J=(0.7, 0.3), sublattice=s3, move=0),
        "tfim_3x3_j2": Model(9, 9, b3, ham=TFIM, J=(1.0, -0.4), h=1.2, sublattice=s3),
    }


@pytest.mark.parametrize("name", list(models().keys()))
@pytest.mark.parametrize("cplx", [False, True])
def test_local_energy_row_identity(name, cplx):
    m = models()[name]
    N, M = m.n_sites, m.n_hidden
    p = synth.rbm_params(N, M, cplx, sigma=0.25, seed=21)
    confs = lattice.all_configs(N)
    psi = np.exp(rbm.log_psi(p, confs, N, M))
    Hpsi = exact.sparse_hamiltonian(m) @ psi
    rng = np.random.default_rng(5)
    rows = rng.choice(confs.shape[0], size=min(64, confs.shape[0]), replace=False)
    el = hamiltonian.local_energy(m, p, confs[rows])
    assert np.allclose(el, Hpsi[rows] / psi[rows], rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("cplx", [False, True])
def test_average_local_energy_is_exact_energy(cplx):
    m = models()["heis8_marshall"]
    p = synth.rbm_params(m.n_sites, m.n_hidden, cplx, sigma=0.3, seed=22)
    confs, pi = exact.exact_probabilities(m, p)
    el = hamiltonian.local_energy(m, p, confs)
    assert abs(pi @ el - exact.exact_energy(m, p)) < 1e-12


def test_uniform_psi_and_zero_coupling():
    b, sub = lattice.hypercube(6, 1)
    m = Model(6, 3, b, ham=TFIM, J=(0.0, 0.0), h=0.9)
    p = np.zeros(rbm.n_params(6, 3))
    s = synth.spin_configs(20, 6, seed=3)
    assert np.allclose(hamiltonian.local_energy(m, p, s), -0.9 * 6, atol=1e-14)
    mh = Model(6, 3, b, ham=HEISENBERG, J=(1.0, 0.0), sublattice=sub, marshall=True)
    el = hamiltonian.local_energy(mh, p, s)
    for k in range(s.shape[0]):
        H = exact.dense_hamiltonian(mh)
        idx = int("".join("0" if x > 0 else "1" for x in s[k]), 2)
        assert abs(el[k] - H[idx].sum()) < 1e-12
