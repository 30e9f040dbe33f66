"""GPU parity of supervised learning (Sec. 2.2.3: the negative log overlap of Eq. 1 and
the update of Eq. 2) against oracle/supervised.py: the cumulative target weights, the
direct draws from |t|^2 on the same Philox stream (indices bit-exact, up to draws the
oracle flags as near-ties), one step's loss and parameter update on the same samples,
and the paper's example run (TFIM ring, N = 10, RBM with 20 hidden units, ED target)."""
import numpy as np
import pytest
import torch

import cases
from oracle import exact, hamiltonian as oh, lattice, rbm, rbm_symm, supervised as osup

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def tfim10_target():
    bonds, sub = lattice.hypercube(10, 1)
    om = oh.Model(10, 20, bonds, ham=0, J=(1.0, 0.0), h=1.0, marshall=False, sublattice=sub,
                  move=0)
    _, v = exact.ground_state(om)
    return lattice.all_configs(10), np.log(v.real)


def tfim10_model(lib):
    bonds, sub = lib.nqs_hypercube(10, 1, False)
    return lib.Model(10, 20, bonds, ham=0, J=(1.0, 0.0), h=1.0, marshall=False,
                     sublattice=sub, move=0, is_complex=False, prec=0)


@pytest.mark.parametrize("cplx", [False, True])
def test_target_cdf_and_draws_match_oracle(lib, cplx):
    name = "tfim10_real_f64" if not cplx else "heis40_cplx_f64"
    m, om = cases.build(lib, name)
    rng = np.random.default_rng(21)
    ns = 1000                                    # a training set that is not a power of two
    states = rng.choice(np.array([-1, 1], dtype=np.int8), size=(ns, om.n_sites))
    lt = rng.normal(0, 1.5, ns) + (1j * rng.uniform(-3, 3, ns) if cplx else 0)
    cdf = m.target_cdf(to_dev(lt))
    cdf_o = osup.target_cdf(lt)
    assert np.abs(cdf.cpu().numpy() - cdf_o).max() <= 1e-13 * cdf_o[-1]
    n = 20011
    sig, ltd, idx = m.target_draw(cdf, to_dev(states), to_dev(lt), n, seed=99, counter=7)
    idx_o = osup.draw(cdf_o, n, seed=99, counter=7)
    ties = set(osup.near_ties(cdf_o, n, seed=99, counter=7).tolist())
    idx = idx.cpu().numpy()
    differ = np.nonzero(idx != idx_o)[0]
    assert set(differ.tolist()) <= ties
    assert np.array_equal(sig.cpu().numpy(), states[idx])
    assert np.array_equal(ltd.cpu().numpy(), lt[idx])


@pytest.mark.parametrize("name", ["tfim10_real_f64", "heis40_cplx_f64", "j1j2_4x4_cplx_f64",
                                  "heis40_cplx_f32", "tfim37_real_f32", "heis6x6_cplx_f32",
                                  "heis4x4_cplx_f32_m1024"])
def test_overlap_step_matches_oracle(lib, name):
    """Loss and update of one step on the same samples and log targets; the targets are
    a random state, so R = psi / t spreads over orders of magnitude."""
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=5)
    rng = np.random.default_rng(6)
    n = 3001
    ch = torch.empty((n, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=3)
    sig = ch.cpu().numpy()
    lt = rng.normal(0, 0.8, n) + (1j * rng.uniform(-np.pi, np.pi, n) if m.is_complex else 0)
    pd = to_dev(p.copy())
    lr = 0.05
    info = m.overlap_step(pd, ch, to_dev(lt), lr)
    po = cases.oracle_params(name, p)
    p_new, loss, g = osup.rbm_step(po, sig, lt, om.n_sites, om.n_hidden, lr)
    tol = cases.tol(name)
    assert info["status"] == lib.OK
    assert abs(info["loss"] - loss) <= tol * max(1.0, abs(loss))
    assert abs(info["grad_norm"] - np.linalg.norm(g)) <= tol * np.linalg.norm(g)
    got = pd.cpu().numpy().astype(np.complex128 if m.is_complex else np.float64)
    # the update in the parameters' own precision: one rounding of p plus lr times the
    # gradient's tolerance
    ulp = 0.0 if m.prec == 0 else 2.0 ** -24 * np.abs(po).max()
    assert np.abs(got - p_new).max() <= lr * tol * np.abs(g).max() + ulp


def test_overlap_step_symmetric_rbm(lib):
    """The symmetric RBM: the gradient of its own parameters (the sums over the copies)."""
    N, alpha = 20, 2
    bonds, sub = lib.nqs_hypercube(N, 1, False)
    perm = lib.nqs_hypercube_translations(N, 1)
    m = lib.Model(N, alpha * N, bonds, ham=1, J=(1.0, 0.0), h=0.0, marshall=True,
                  sublattice=sub, move=1, is_complex=True, prec=0, symm=perm)
    rng = np.random.default_rng(8)
    P = rbm_symm.n_params(N, alpha)
    p = rng.normal(0, 0.1, P) + 1j * rng.normal(0, 0.1, P)
    n = 777
    ch = torch.empty((n, N), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=4)
    sig = ch.cpu().numpy()
    lt = rng.normal(0, 0.5, n) + 1j * rng.uniform(-np.pi, np.pi, n)
    pd = to_dev(p.copy())
    info = m.overlap_step(pd, ch, to_dev(lt), 0.1)
    perm_np = perm.cpu().numpy() if hasattr(perm, "cpu") else np.asarray(perm)
    lp = rbm_symm.log_psi(p, sig, N, alpha, perm_np)
    O = rbm_symm.log_derivatives(p, sig, N, alpha, perm_np)
    loss, g, _ = osup.estimator(lp, lt, O)
    assert abs(info["loss"] - loss) <= 1e-10 * max(1.0, abs(loss))
    assert np.abs(pd.cpu().numpy() - (p - 0.1 * g)).max() <= 1e-10 * 0.1 * np.abs(g).max()


def test_overlap_step_nonfinite_leaves_parameters(lib):
    m, om = cases.build(lib, "heis40_cplx_f32")
    p = to_dev(cases.params("heis40_cplx_f32"))
    p0 = p.clone()
    ch = torch.empty((64, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=3)
    lt = np.zeros(64, dtype=np.complex128)
    lt[17] = np.nan
    info = m.overlap_step(p, ch, to_dev(lt), 0.1)
    assert info["status"] == lib.ENONFINITE
    assert torch.equal(p, p0)


def test_paper_example_tfim10_supervised(lib):
    """The example of Sec. 3 (supervised learning of the TFIM ground state, N = 10, 20
    hidden units, parameters N(0, 0.01^2) with seed 1234, batches of 400 direct draws),
    with the update of Eq. 2 at learning rate 0.1: the first 20 steps follow the oracle
    replaying the same draws to 1e-10, and after 300 steps the exact overlap exceeds 0.97."""
    m = tfim10_model(lib)
    states, lt = tfim10_target()
    p0 = np.random.default_rng(1234).normal(0, 0.01, rbm.n_params(10, 20))
    pd = to_dev(p0.copy())
    st_d, lt_d = to_dev(states), to_dev(lt)
    cdf = m.target_cdf(lt_d)
    cdf_o = osup.target_cdf(lt)
    po = p0.copy()
    for it in range(300):
        sig, ltb, idx = m.target_draw(cdf, st_d, lt_d, 400, seed=1234, counter=it)
        info = m.overlap_step(pd, sig, ltb, 0.1)
        assert info["status"] == lib.OK
        if it < 20:
            io = osup.draw(cdf_o, 400, seed=1234, counter=it)
            assert np.array_equal(idx.cpu().numpy(), io)
            po, loss, _ = osup.rbm_step(po, states[io], lt[io], 10, 20, 0.1)
            assert abs(info["loss"] - loss) <= 1e-10 * max(1.0, loss)
            assert np.abs(pd.cpu().numpy() - po).max() <= 1e-10 * np.abs(po).max()
    L, _ = osup.rbm_exact(pd.cpu().numpy(), lt, 10, 20)
    assert np.exp(-L) > 0.97, np.exp(-L)
