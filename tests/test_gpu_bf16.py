"""GPU parity of the BF16 precision form: the library's BF16 model against the oracle
running the same quantised model (W rounded to bfloat16, tanh(theta) rounded in the
Jacobian contractions). Arithmetic is FP32, so the FP32 tolerance (1e-5 relative)
applies; the energy of the quantised model is also compared with the unquantised FP64
model (2e-3 relative)."""
import numpy as np
import pytest
import torch

import cases
from oracle import hamiltonian as oh, rbm as orbm, sampler as osamp, sr as osr

pytestmark = pytest.mark.gpu

DEV = "cuda"
NAMES = list(cases.BF16)


def tanh_tie_ulps(pe, s, N, M, margin=2.0 ** -9):
    """Entries of tanh(theta) within `margin` bfloat16 ulps of a rounding midpoint: there
    the library (theta and tanh in FP32) may round to the other neighbour than the oracle
    (FP64). FP32 accumulation of theta over N ~ 40 terms of size ~0.05 errs by ~4e-7,
    about 2^-12 of a bfloat16 ulp at |tanh| ~ 0.3, so the margin is ~10x that. Returns
    |ulp| at those entries, 0 elsewhere, [n, M]."""
    t = np.tanh(orbm.theta(pe, s, N, M))

    def comp(x):
        m, e = np.frexp(x)
        y = np.abs(m) * 256.0
        near = np.abs(y - np.floor(y) - 0.5) < margin
        return np.where(near, np.ldexp(1.0, e - 8), 0.0)

    if np.iscomplexobj(t):
        return np.hypot(comp(t.real), comp(t.imag))
    return comp(t)


def tie_bounds(pe, s, N, M, u=None, v=None):
    """Worst-case effect of the tie entries on O v (per sample) and O^dagger u (per
    parameter): each tie may move its tanh(theta) entry by one bfloat16 ulp."""
    D = tanh_tie_ulps(pe, s, N, M)
    out = []
    if v is not None:
        a_, b_, W = v[:N], v[N:N + M], v[N + M:].reshape(M, N)
        fac = np.abs(b_[None, :] + s.astype(np.float64) @ W.T)        # [n, M]
        out.append((D * fac).sum(axis=1))
    if u is not None:
        g = D.T @ np.abs(u)                                            # [M]
        out.append(np.concatenate([np.zeros(N), g, np.repeat(g, N)]))
    return out, int((D > 0).sum())


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def wrap(d):
    return np.angle(np.exp(1j * d))


@pytest.mark.parametrize("name", NAMES)
def test_bf16_log_psi(lib, name):
    """log psi is evaluated in double from the quantised weights."""
    m, om = cases.build(lib, name)
    p = cases.params(name)
    s = cases.configs(name, 301, seed=5)
    got = m.log_psi(to_dev(p), to_dev(s)).cpu().numpy()
    exp = orbm.log_psi(cases.oracle_params(name, p), s, om.n_sites, om.n_hidden)
    assert np.all(np.abs(np.real(got) - np.real(exp)) <= 1e-10 * np.maximum(1, np.abs(np.real(exp))))
    if m.is_complex:
        assert np.all(np.abs(wrap(np.imag(got) - np.imag(exp))) <= 1e-10 * np.maximum(1, np.abs(np.imag(exp))))


@pytest.mark.parametrize("name", NAMES)
def test_bf16_local_energy(lib, name):
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=11)
    s = cases.configs(name, 203, seed=6)
    got = m.local_energy(to_dev(p), to_dev(s)).cpu().numpy()
    exp = oh.local_energy(om, cases.oracle_params(name, p), s)
    scale = max(1.0, np.abs(exp).max())
    assert np.abs(got - exp).max() <= cases.tol(name) * scale


@pytest.mark.parametrize("name", NAMES)
def test_bf16_energy_against_unquantised_model(lib, name):
    """Mean local energy of the quantised model over |psi|^2-distributed samples against
    the FP64 unquantised model on the same samples: within 2e-3 relative."""
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=0.5, seed=12)
    C = 256
    ch = torch.empty((C, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=5)
    smp, el = m.sample(to_dev(p), ch, 8, 40, seed=5, counter=0, with_eloc=True)
    flat = smp.reshape(-1, om.n_sites).cpu().numpy()
    e_full = oh.local_energy(om, p.astype(np.complex128 if m.is_complex else np.float64), flat)
    E_q = np.real(el.cpu().numpy().mean())
    E_f = np.real(e_full.mean())
    assert abs(E_q - E_f) <= 2e-3 * abs(E_f), (E_q, E_f)


@pytest.mark.parametrize("name", NAMES)
def test_bf16_sampling(lib, name):
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=31)
    C, n_sweeps, n_discard = 24, 6, 3
    ch = torch.empty((C, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=1234)
    init = ch.cpu().numpy().copy()
    smp, _ = m.sample(to_dev(p), ch, n_sweeps, n_discard, seed=1234, counter=17)
    ties = []
    exp, last, _ = osamp.sample(om, cases.oracle_params(name, p), init, n_sweeps, n_discard,
                                seed=1234, counter=17, record_ties=ties, tie_margin=1e-4)
    got = smp.cpu().numpy()
    cases.compare_chains(got, exp, ties, n_discard)


@pytest.mark.parametrize("name", NAMES)
def test_bf16_jvp_vjp(lib, name):
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=21)
    n = 517
    s = cases.configs(name, n, seed=7)
    rng = np.random.default_rng(3)
    P = m.n_params
    u = rng.normal(size=n) + (1j * rng.normal(size=n) if m.is_complex else 0)
    v = rng.normal(size=P) + (1j * rng.normal(size=P) if m.is_complex else 0)
    vjp, jvp = m.log_psi_grad(to_dev(p), to_dev(s), u=to_dev(u), v=to_dev(v))
    O = orbm.log_derivatives(cases.oracle_params(name, p), s, om.n_sites, om.n_hidden,
                             cases.round_tanh(name))
    if not m.is_complex:
        O = O.real
    ej, ev = O @ v, O.conj().T @ u
    t = cases.tol(name)
    (bj, bv), ties = tie_bounds(cases.oracle_params(name, p), s, om.n_sites, om.n_hidden, u, v)
    assert ties < 0.02 * n * om.n_hidden + 5
    assert np.all(np.abs(jvp.cpu().numpy() - ej) <= t * np.abs(ej).max() + 1.01 * bj)
    assert np.all(np.abs(vjp.cpu().numpy() - ev) <= t * np.abs(ev).max() + 1.01 * bv)


@pytest.mark.parametrize("name,n", [("heis40_cplx_bf16", 1000), ("j1j2_4x4_cplx_bf16", 333),
                                    ("tfim37_real_bf16", 517)])
def test_bf16_sr_matvec(lib, name, n):
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=0.3, seed=61)
    s = cases.configs(name, n, seed=10)
    st = to_dev(s)
    ws = m.sr_prepare(to_dev(p), st)
    rng = np.random.default_rng(62)
    v = rng.normal(size=m.n_params) + (1j * rng.normal(size=m.n_params) if m.is_complex else 0)
    got = m.sr_matvec(st, ws, to_dev(v), diag_shift=0.01).cpu().numpy()
    O = orbm.log_derivatives(cases.oracle_params(name, p), s, om.n_sites, om.n_hidden,
                             cases.round_tanh(name))
    if not m.is_complex:
        O = O.real
    exp = osr.s_matrix(O) @ v + 0.01 * v
    y = O @ v
    scale = np.abs(O.conj().T @ y).max() / n
    # ties: a moved entry changes y_s (first bound) and the column it enters in O^dagger
    # (second bound, with u = y - mean y)
    (by,), _ = tie_bounds(cases.oracle_params(name, p), s, om.n_sites, om.n_hidden, v=v)
    (bu,), ties = tie_bounds(cases.oracle_params(name, p), s, om.n_sites, om.n_hidden,
                             u=np.abs(y - y.mean()) + by)
    extra = (bu + np.abs(O).T @ by) / n
    assert np.all(np.abs(got - exp) <= cases.tol(name) * scale + 1.01 * extra)


@pytest.mark.parametrize("name", NAMES)
def test_bf16_sr_step(lib, name):
    """12 CG products with FP32 arithmetic on the quantised operands: the step agrees
    with the oracle's to 1e-4 of its size (as for the FP32 form)."""
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=0.3, seed=52)
    n = 640
    s = cases.configs(name, n, seed=9)
    pe = cases.oracle_params(name, p)
    el = oh.local_energy(om, pe, s)
    pt = to_dev(p.copy())
    m.sr_step(pt, to_dev(s), to_dev(el), lr=0.05, diag_shift=0.01, cg_tol=0.0, cg_maxiter=12)
    p_new, _ = osr.sr_step(om, pe, s, el, lr=0.05, diag_shift=0.01, cg_tol=0.0, cg_maxiter=12,
                           round_tanh=cases.round_tanh(name))
    step_o = p_new - pe
    p_start = np.asarray(p).astype(pe.dtype)
    step_g = pt.cpu().numpy().astype(pe.dtype) - p_start
    assert np.abs(step_g - step_o).max() <= 1e-4 * np.abs(step_o).max() + 1e-7
