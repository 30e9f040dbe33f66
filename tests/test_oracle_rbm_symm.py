"""Pins of the oracle symmetric RBM: invariance under the lattice translations, hidden-unit
marginalisation, equality with the expanded plain RBM, finite differences of O_k, and the
SR force against finite differences of the exact energy."""
import numpy as np
import pytest

import synth
from oracle import exact, lattice, rbm, rbm_symm, sr
from oracle.hamiltonian import HEISENBERG, TFIM, Model


def params(N, alpha, cplx, sigma, seed):
    rng = np.random.default_rng(seed)
    P = rbm_symm.n_params(N, alpha)
    p = rng.normal(0.0, sigma, P)
    if cplx:
        p = p + 1j * rng.normal(0.0, sigma, P)
    return p


@pytest.mark.parametrize("L,ndim", [(6, 1), (3, 2), (4, 2)])
def test_translations_form_a_group(L, ndim):
    perm = rbm_symm.translations(L, ndim)
    G, N = perm.shape
    assert G == N == L ** ndim
    assert np.array_equal(perm[0], np.arange(N))              # identity
    rows = {tuple(r) for r in perm}
    assert len(rows) == G
    for g in range(G):
        assert sorted(perm[g]) == list(range(N))               # permutations
        for h in range(G):
            assert tuple(perm[h][perm[g]]) in rows             # closure


@pytest.mark.parametrize("cplx", [False, True])
def test_invariance_under_translations(cplx):
    N, alpha = 8, 2
    perm = rbm_symm.translations(N, 1)
    p = params(N, alpha, cplx, 0.4, 3)
    s = synth.spin_configs(20, N, seed=4)
    lp = rbm_symm.log_psi(p, s, N, alpha, perm)
    for h in range(N):
        th = rbm_symm.log_psi(p, s[:, perm[h]], N, alpha, perm)
        assert np.allclose(np.exp(th), np.exp(lp), rtol=1e-12)
    # a plain RBM of the same size is not invariant (the pin has teeth)
    q = synth.rbm_params(N, alpha * N, cplx, sigma=0.4, seed=5)
    r0 = rbm.log_psi(q, s, N, alpha * N)
    r1 = rbm.log_psi(q, s[:, perm[1]], N, alpha * N)
    assert np.abs(r0 - r1).max() > 1e-3


@pytest.mark.parametrize("cplx", [False, True])
def test_hidden_sum_and_expansion(cplx):
    N, alpha = 4, 2
    perm = rbm_symm.translations(N, 1)
    p = params(N, alpha, cplx, 0.5, 6)
    s = lattice.all_configs(N)
    a = rbm_symm.log_psi(p, s, N, alpha, perm)
    b = rbm_symm.log_psi_hidden_sum(p, s, N, alpha, perm)
    assert np.allclose(a.real, b.real, atol=1e-12)
    assert np.allclose(np.angle(np.exp(1j * (a.imag - b.imag))), 0, atol=1e-12)
    pe = rbm_symm.expand(p, N, alpha, perm)
    c = rbm.log_psi(pe, s, N, alpha * N)
    assert np.allclose(np.exp(a), np.exp(c), rtol=1e-13)
    # 2D: the expansion of a 3x3 lattice
    perm2 = rbm_symm.translations(3, 2)
    p2 = params(9, 1, cplx, 0.3, 7)
    s2 = synth.spin_configs(30, 9, seed=8)
    assert np.allclose(np.exp(rbm_symm.log_psi(p2, s2, 9, 1, perm2)),
                       np.exp(rbm.log_psi(rbm_symm.expand(p2, 9, 1, perm2), s2, 9, 9)), rtol=1e-13)


@pytest.mark.parametrize("cplx", [False, True])
def test_log_derivatives_match_finite_differences(cplx):
    N, alpha = 6, 2
    perm = rbm_symm.translations(N, 1)
    p = params(N, alpha, cplx, 0.3, 9)
    s = synth.spin_configs(7, N, seed=10)
    O = rbm_symm.log_derivatives(p, s, N, alpha, perm)
    eps = 1e-6
    for k in range(p.size):
        dp = np.zeros_like(p)
        dp[k] = eps
        fd = (rbm_symm.log_psi(p + dp, s, N, alpha, perm)
              - rbm_symm.log_psi(p - dp, s, N, alpha, perm)) / (2 * eps)
        assert np.allclose(fd, O[:, k], rtol=1e-7, atol=1e-8), k


def test_force_matches_energy_finite_differences():
    N, alpha = 6, 2
    b, sub = lattice.hypercube(N, 1)
    perm = rbm_symm.translations(N, 1)
    m = Model(N, alpha * N, b, ham=HEISENBERG, J=(1.0, 0.0), sublattice=sub, marshall=True,
              is_complex=True)
    p = params(N, alpha, True, 0.3, 11)

    def energy(q):
        return exact.exact_energy(m, rbm_symm.expand(q, N, alpha, perm)).real

    confs, pi = exact.exact_probabilities(m, rbm_symm.expand(p, N, alpha, perm))
    O = rbm_symm.log_derivatives(p, confs, N, alpha, perm)
    from oracle import hamiltonian
    el = hamiltonian.local_energy(m, rbm_symm.expand(p, N, alpha, perm), confs)
    F = sr.force(O, el, pi)
    eps = 1e-5
    for k in range(p.size):
        d = np.zeros_like(p)
        d[k] = eps
        g_re = (energy(p + d) - energy(p - d)) / (2 * eps)
        g_im = (energy(p + 1j * d) - energy(p - 1j * d)) / (2 * eps)
        assert abs(g_re - 2 * F[k].real) < 1e-6 * max(1.0, abs(g_re)), k
        assert abs(g_im - 2 * F[k].imag) < 1e-6 * max(1.0, abs(g_im)), k
