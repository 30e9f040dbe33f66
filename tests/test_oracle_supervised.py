"""Pins of the supervised-learning oracle (Sec. 2.2.3, Eq. 1 and Eq. 2) against what the
definition and the mathematics fix: the full-sum overlap, finite differences, the exact
zero of the loss, the Cauchy-Schwarz bound, the target distribution of the draws, and
the ground state of the transverse-field Ising ring."""
import numpy as np
import pytest
from scipy import stats

from oracle import exact, hamiltonian as oh, lattice, rbm, supervised as osup


def rand_params(rng, N, M, cplx, s):
    P = rbm.n_params(N, M)
    p = rng.normal(0, s, P)
    if cplx:
        p = p + 1j * rng.normal(0, s, P)
    return p


def rand_target(rng, N, cplx):
    """log t of a random state over all 2^N configurations."""
    lt = rng.normal(0, 0.7, 2 ** N)
    if cplx:
        lt = lt + 1j * rng.uniform(-np.pi, np.pi, 2 ** N)
    return lt


@pytest.mark.parametrize("cplx", [False, True])
def test_weighted_estimator_over_all_states_is_the_definition(cplx):
    """With every configuration weighted by the exact |t|^2 the estimator is Eq. 1 and its
    derivative computed from the full sums <t|psi>, <psi|psi>, <t|t>."""
    rng = np.random.default_rng(3)
    N, M = 6, 4
    p = rand_params(rng, N, M, cplx, 0.3)
    lt = rand_target(rng, N, cplx)
    confs = lattice.all_configs(N)
    lp = rbm.log_psi(p, confs, N, M)
    O = rbm.log_derivatives(p, confs, N, M)
    w = np.exp(2 * lt.real)
    loss, g, _ = osup.estimator(lp, lt, O, weights=w, real_params=not cplx)
    # the definition, term by term, in the plain amplitudes
    psi, t = np.exp(lp), np.exp(lt)
    ov = abs(np.sum(np.conj(t) * psi)) ** 2 / (np.sum(abs(t) ** 2) * np.sum(abs(psi) ** 2))
    assert abs(loss - (-np.log(ov))) <= 1e-12
    assert abs(osup.exact_loss(lp, lt) - (-np.log(ov))) <= 1e-12
    ge = osup.exact_gradient(lp, lt, O, real_params=not cplx)
    assert np.abs(g - ge).max() <= 1e-12 * np.abs(ge).max()


@pytest.mark.parametrize("cplx", [False, True])
def test_gradient_is_the_finite_difference_of_the_loss(cplx):
    """dL/dRe(alpha_k) = 2 Re g_k and dL/dIm(alpha_k) = 2 Im g_k (g = dL/dconj(alpha))."""
    rng = np.random.default_rng(5)
    N, M = 5, 3
    p = rand_params(rng, N, M, cplx, 0.4)
    lt = rand_target(rng, N, cplx)
    L0, g = osup.rbm_exact(p, lt, N, M)
    eps = 1e-6
    for k in rng.choice(len(p), 8, replace=False):
        for d in ((1.0, 1j) if cplx else (1.0,)):
            e = np.zeros(len(p), dtype=p.dtype)
            e[k] = d * eps
            fd = (osup.rbm_exact(p + e, lt, N, M)[0] - osup.rbm_exact(p - e, lt, N, M)[0]) / (2 * eps)
            exp = 2 * (g[k].real if d == 1.0 else np.imag(g[k]))
            assert abs(fd - exp) <= 1e-6 * max(1.0, np.abs(g).max()), (k, d, fd, exp)


def test_loss_vanishes_when_psi_is_proportional_to_the_target():
    rng = np.random.default_rng(9)
    N, M = 6, 5
    p = rand_params(rng, N, M, True, 0.3)
    confs = lattice.all_configs(N)
    lt = rbm.log_psi(p, confs, N, M) + (0.7 - 1.3j)
    L, g = osup.rbm_exact(p, lt, N, M)
    assert abs(L) <= 1e-12 and np.abs(g).max() <= 1e-12
    idx = rng.integers(0, 2 ** N, 50)
    _, loss, gs = osup.rbm_step(p, confs[idx], lt[idx], N, M, lr=0.1)
    assert abs(loss) <= 1e-12 and np.abs(gs).max() <= 1e-12


def test_loss_is_nonnegative_and_sgd_lowers_it():
    """Cauchy-Schwarz bounds the overlap by one; a small step along -g lowers the loss."""
    rng = np.random.default_rng(11)
    N, M = 6, 6
    lt = rand_target(rng, N, True)
    for _ in range(5):
        p = rand_params(rng, N, M, True, 0.5)
        L0, g = osup.rbm_exact(p, lt, N, M)
        assert L0 >= 0
        L1, _ = osup.rbm_exact(p - 1e-3 * g, lt, N, M)
        assert L1 < L0


def test_draws_follow_the_target_distribution():
    rng = np.random.default_rng(13)
    N = 6
    lt = rand_target(rng, N, True)
    cdf = osup.target_cdf(lt)
    n = 200000
    idx = osup.draw(cdf, n, seed=77, counter=4)
    assert idx.min() >= 0 and idx.max() < 2 ** N
    p = np.exp(2 * lt.real)
    p /= p.sum()
    counts = np.bincount(idx, minlength=2 ** N)
    chi2 = np.sum((counts - n * p) ** 2 / (n * p))
    assert stats.chi2.sf(chi2, 2 ** N - 1) > 1e-3
    # different counters give different draws
    assert not np.array_equal(idx[:100], osup.draw(cdf, 100, seed=77, counter=5))


def test_tfim_ground_state_target():
    """The ED target of the paper's example (TFIM ring, N = 10, h = 1): its energy is the
    free-fermion closed form, its amplitudes are positive (so log t is real), and the RBM
    can only lower the loss toward it from the random start."""
    bonds, sub = lattice.hypercube(10, 1)
    om = oh.Model(10, 10, bonds, ham=0, J=(1.0, 0.0), h=1.0, marshall=False, sublattice=sub,
                  move=0)
    e0, v = exact.ground_state(om)
    assert abs(e0 - exact.tfim_ground_energy(10)) <= 1e-10
    assert np.all(v.real > 0) and np.abs(v.imag).max() <= 1e-12
    lt = np.log(v.real)
    rng = np.random.default_rng(1234)
    p = rng.normal(0, 0.01, rbm.n_params(10, 20))
    L0, g = osup.rbm_exact(p, lt, 10, 20)
    assert 0 < L0 < 2   # overlap of the near-uniform start with the ground state ~ 0.34
    assert osup.rbm_exact(p - 0.05 * g, lt, 10, 20)[0] < L0
