"""Pins of the oracle SR: force against finite differences of the exact energy, the S
quadratic form against the finite-difference tangent vector of psi, CG against a dense
solve, exact-expectation SR descending to the exact ground energy."""
import numpy as np
import pytest

import synth
from oracle import exact, hamiltonian, lattice, rbm, sr
from oracle.hamiltonian import HEISENBERG, TFIM, Model


def small_model(cplx=True):
    b, sub = lattice.hypercube(5, 1)
    return Model(5, 3, b, ham=TFIM, J=(1.0, 0.0), h=0.7, sublattice=sub, is_complex=cplx)


def exact_force(m, p):
    confs, pi = exact.exact_probabilities(m, p)
    O = rbm.log_derivatives(p, confs, m.n_sites, m.n_hidden)
    el = hamiltonian.local_energy(m, p, confs)
    return sr.force(O, el, pi)


@pytest.mark.parametrize("cplx", [False, True])
def test_force_matches_energy_finite_differences(cplx):
    m = small_model(cplx)
    p = synth.rbm_params(m.n_sites, m.n_hidden, cplx, sigma=0.3, seed=41)
    F = exact_force(m, p)
    eps = 1e-5
    for k in range(p.size):
        d = np.zeros_like(p); d[k] = eps
        g_re = (exact.exact_energy(m, p + d).real - exact.exact_energy(m, p - d).real) / (2 * eps)
        assert abs(g_re - 2 * F[k].real) < 1e-6 * max(1.0, abs(g_re)), k
        if cplx:
            g_im = (exact.exact_energy(m, p + 1j * d).real - exact.exact_energy(m, p - 1j * d).real) / (2 * eps)
            assert abs(g_im - 2 * F[k].imag) < 1e-6 * max(1.0, abs(g_im)), k


@pytest.mark.parametrize("cplx", [False, True])
def test_s_quadratic_form_matches_tangent_vector(cplx):
    m = small_model(cplx)
    N, M = m.n_sites, m.n_hidden
    p = synth.rbm_params(N, M, cplx, sigma=0.3, seed=42)
    confs, pi = exact.exact_probabilities(m, p)
    S = sr.s_matrix(rbm.log_derivatives(p, confs, N, M), pi)
    if not cplx:
        S = S.real
    for seed in range(4):
        v = synth.random_vector(p.size, cplx, 100 + seed)
        eps = 1e-6
        psi = np.exp(rbm.log_psi(p, confs, N, M))
        dpsi = (np.exp(rbm.log_psi(p + eps * v, confs, N, M)) - np.exp(rbm.log_psi(p - eps * v, confs, N, M))) / (2 * eps)
        nn = np.vdot(psi, psi).real
        q = np.vdot(dpsi, dpsi).real / nn - abs(np.vdot(psi, dpsi)) ** 2 / nn ** 2
        assert abs(np.vdot(v, S @ v).real - q) < 1e-7 * abs(q)


def test_cg_matches_dense_solve():
    m = small_model(True)
    p = synth.rbm_params(m.n_sites, m.n_hidden, True, sigma=0.3, seed=43)
    smp = synth.spin_configs(200, m.n_sites, seed=44)
    O = rbm.log_derivatives(p, smp, m.n_sites, m.n_hidden)
    el = hamiltonian.local_energy(m, p, smp)
    F = sr.force(O, el)
    A = sr.s_matrix(O) + 0.01 * np.eye(p.size)
    x, it, res = sr.cg(lambda v: A @ v, F, 1e-13, 1000)
    assert res <= 1e-13
    xd = np.linalg.solve(A, F)
    assert np.linalg.norm(x - xd) < 1e-9 * np.linalg.norm(xd)
    # maxiter cut
    x1, it1, res1 = sr.cg(lambda v: A @ v, F, 1e-13, 3)
    assert it1 == 3 and res1 > 1e-13


def test_exact_sr_descends_to_ground_energy():
    b, sub = lattice.hypercube(6, 1)
    m = Model(6, 12, b, ham=TFIM, J=(1.0, 0.0), h=1.0, sublattice=sub)
    p = synth.rbm_params(6, 12, False, sigma=0.01, seed=1234)
    e0 = exact.tfim_ground_energy(6, 1.0, 1.0)
    energies = []
    for it in range(150):
        p, info = sr.exact_sr_step(m, p, lr=0.1, diag_shift=0.01)
        energies.append(info["energy"].real)
    assert energies[-1] < energies[0]
    assert np.all(np.diff(energies[5:]) < 1e-9)
    assert abs(energies[-1] - e0) / abs(e0) < 2e-3


def test_stats_hand_built_chain_means():
    # chain c holds c + d_s with sweep offsets d_s summing to zero: the chain means are
    # exactly 0, 1, ..., C-1, so err = sqrt(var(0..C-1, unbiased) / C) = sqrt((C + 1) / 12)
    C, S = 7, 4
    d = np.array([0.5, -1.25, 0.25, 0.5])
    e = np.arange(C)[None, :] + d[:, None]          # [sweeps, chains]
    mean, var, err = sr.stats(e.ravel(), n_chains=C)
    assert abs(mean - (C - 1) / 2.0) < 1e-14
    # population variance: between-chain part (C^2 - 1) / 12 plus the sweep offsets
    assert abs(var - ((C * C - 1) / 12.0 + np.mean(d * d))) < 1e-13
    assert abs(err - np.sqrt((C + 1) / 12.0)) < 1e-14
    # the transposed layout (chains as rows) has different chain means
    assert abs(sr.stats(e.T.ravel(), n_chains=C)[2] - err) > 0.1
    # complex energies: the error bar is that of the real part
    _, _, err_c = sr.stats(e.ravel() + 1j * np.arange(C * S), n_chains=C)
    assert abs(err_c - err) < 1e-14
    # no chain count: every sample is a chain
    x = np.array([1.0, 2.0, 4.0, 7.0])
    assert abs(sr.stats(x)[2] - np.std(x, ddof=1) / 2.0) < 1e-14
    with pytest.raises(ValueError):
        sr.stats(np.ones(6), n_chains=4)


def test_stats_error_bar_is_unbiased():
    # E[err^2] = Var(chain mean) / C = sigma^2 / n for independent samples; a biased
    # (1/C) variance of the chain means would give (C - 1) / C of it
    rng = np.random.default_rng(5)
    C, S, trials, sigma = 4, 3, 20000, 1.7
    e = rng.normal(0.0, sigma, size=(trials, S * C))
    err2 = np.array([sr.stats(row, n_chains=C)[2] ** 2 for row in e])
    ratio = err2.mean() / (sigma ** 2 / (S * C))
    assert abs(ratio - 1.0) < 0.03, ratio
