"""GPU checks of the autograd function over log psi: backward equals O^dagger g from the
oracle's log-derivatives, and central finite differences of the oracle's log psi."""
import numpy as np
import pytest
import torch

import cases
from oracle import rbm as orbm

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("name", ["tfim10_real_f64", "j1j2_4x4_cplx_f64", "heis40_cplx_f32",
                                  "tfim37_real_f32", "heis40_cplx_bf16"])
def test_backward_matches_oracle(lib, name):
    from paper_1904_00031_amd import autograd as nag
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=71)
    n = 301
    s = cases.configs(name, n, seed=13)
    rng = np.random.default_rng(14)
    w = rng.normal(size=n) + (1j * rng.normal(size=n) if m.is_complex else 0)
    pt = to_dev(p).requires_grad_(True)
    lp = nag.log_psi(m, pt, to_dev(s))
    loss = (to_dev(w) * lp).real.sum()
    loss.backward()
    got = pt.grad.cpu().numpy().astype(np.complex128 if m.is_complex else np.float64)
    pe = cases.oracle_params(name, p)
    O = orbm.log_derivatives(pe, s, om.n_sites, om.n_hidden, cases.round_tanh(name))
    if not m.is_complex:
        O = O.real
    # L = Re sum_s w_s log psi_s  =>  dL/dRe z_s + i dL/dIm z_s = conj(w_s)
    exp = O.conj().T @ np.conj(w)
    tol = 1e-10 if cases.CASES[name][9] == 0 else 1e-5
    if cases.CASES[name][9] == 2:
        tol = 2e-3   # rounded tanh rows near bfloat16 midpoints (see the BF16 tests)
    assert np.abs(got - exp).max() <= tol * np.abs(exp).max()


@pytest.mark.parametrize("name", ["j1j2_4x4_cplx_f64", "tfim10_real_f64"])
def test_backward_matches_finite_differences(lib, name):
    from paper_1904_00031_amd import autograd as nag
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=72)
    n = 64
    s = cases.configs(name, n, seed=15)
    rng = np.random.default_rng(16)
    w = rng.normal(size=n) + (1j * rng.normal(size=n) if m.is_complex else 0)
    pt = to_dev(p).requires_grad_(True)
    (to_dev(w) * nag.log_psi(m, pt, to_dev(s))).real.sum().backward()
    got = pt.grad.cpu().numpy()

    def L(q):
        return np.real(w @ orbm.log_psi(q, s, om.n_sites, om.n_hidden))

    eps = 1e-6
    for k in rng.choice(m.n_params, 12, replace=False):
        e = np.zeros(m.n_params, dtype=p.dtype)
        e[k] = eps
        d_re = (L(p + e) - L(p - e)) / (2 * eps)
        fd = d_re
        if m.is_complex:
            d_im = (L(p + 1j * e) - L(p - 1j * e)) / (2 * eps)
            fd = d_re + 1j * d_im
        assert abs(got[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, got[k], fd)


def test_jvp_and_sv_helpers(lib):
    from paper_1904_00031_amd import autograd as nag
    from oracle import sr as osr
    name = "j1j2_4x4_cplx_f64"
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=73)
    s = cases.configs(name, 200, seed=17)
    rng = np.random.default_rng(18)
    v = rng.normal(size=m.n_params) + 1j * rng.normal(size=m.n_params)
    O = orbm.log_derivatives(p, s, om.n_sites, om.n_hidden)
    jv = nag.log_psi_jvp(m, to_dev(p), to_dev(s), to_dev(v)).cpu().numpy()
    assert np.abs(jv - O @ v).max() <= 1e-10 * np.abs(O @ v).max()
    sv = nag.sv_product(m, to_dev(p), to_dev(s), to_dev(v), 0.01).cpu().numpy()
    exp = osr.s_matrix(O) @ v + 0.01 * v
    assert np.abs(sv - exp).max() <= 1e-10 * np.abs(exp).max()
