"""GPU parity on the large lattices (10x10 J1-J2 with 400 hidden units, 16x16 Heisenberg
with 2048 hidden units), FP32 and BF16 forms, on few samples: the oracle evaluates the
same quantities one by one (log psi, local energies, sampled chains, single columns of
the Jacobian products)."""
import numpy as np
import pytest
import torch

import cases
from oracle import hamiltonian as oh, rbm as orbm, sampler as osamp

pytestmark = pytest.mark.gpu

DEV = "cuda"
NAMES = ["j1j2_10x10_cplx_f32", "heis16x16_cplx_f32", "j1j2_10x10_cplx_bf16",
         "heis16x16_cplx_bf16"]


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def wrap(d):
    return np.angle(np.exp(1j * d))


@pytest.mark.parametrize("name", NAMES)
def test_large_log_psi_and_local_energy(lib, name):
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=81)
    pe = cases.oracle_params(name, p)
    n = 6 if om.n_sites > 200 else 16
    s = cases.configs(name, n, seed=19)
    lp = m.log_psi(to_dev(p), to_dev(s)).cpu().numpy()
    elp = orbm.log_psi(pe, s, om.n_sites, om.n_hidden)
    assert np.all(np.abs(lp.real - elp.real) <= 1e-10 * np.maximum(1, np.abs(elp.real)))
    assert np.all(np.abs(wrap(lp.imag - elp.imag)) <= 1e-10 * np.maximum(1, np.abs(elp.imag)))
    el = m.local_energy(to_dev(p), to_dev(s)).cpu().numpy()
    eel = oh.local_energy(om, pe, s)
    assert np.abs(el - eel).max() <= cases.tol(name) * max(1.0, np.abs(eel).max())


@pytest.mark.parametrize("name", NAMES)
def test_large_sampling(lib, name):
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=82)
    C = 8
    ch = torch.empty((C, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=77)
    init = ch.cpu().numpy().copy()
    smp, el = m.sample(to_dev(p), ch, 2, 1, seed=77, counter=3, with_eloc=True)
    ties = []
    exp, _, _ = osamp.sample(om, cases.oracle_params(name, p), init, 2, 1, seed=77, counter=3,
                             record_ties=ties, tie_margin=1e-4)
    got = smp.cpu().numpy()
    cases.compare_chains(got, exp, ties, 1)
    # local energies of the last recorded sweep, fused or not
    rows = got[-1]
    eel = oh.local_energy(om, cases.oracle_params(name, p), rows)
    gel = el.cpu().numpy().reshape(2, C)[-1]
    assert np.abs(gel - eel).max() <= cases.tol(name) * max(1.0, np.abs(eel).max())


@pytest.mark.parametrize("name", NAMES)
def test_large_jacobian_and_sv_sampled(lib, name):
    """O v on every sample and selected entries of O^dagger u and of S v, each entry
    from its own oracle column."""
    m, om = cases.build(lib, name)
    N, M = om.n_sites, om.n_hidden
    p = cases.params(name, theta=0.3, seed=83)
    pe = cases.oracle_params(name, p)
    rt = cases.round_tanh(name)
    n = 96
    s = cases.configs(name, n, seed=20)
    rng = np.random.default_rng(21)
    P = m.n_params
    u = rng.normal(size=n) + 1j * rng.normal(size=n)
    v = rng.normal(size=P) + 1j * rng.normal(size=P)
    vjp, jvp = m.log_psi_grad(to_dev(p), to_dev(s), u=to_dev(u), v=to_dev(v))
    ej = np.concatenate([orbm.jvp(pe, s[i:i + 8], v, N, M, rt) for i in range(0, n, 8)])
    ks = np.unique(np.concatenate([[0, N - 1, N, N + M - 1, P - 1], rng.integers(0, P, 40)]))
    ev = orbm.vjp_entries(pe, s, u, ks, N, M, rt)
    slack = 2e-3 if rt is not None else 0.0   # bfloat16 rounding ties of tanh(theta)
    t = cases.tol(name) + slack
    assert np.abs(jvp.cpu().numpy() - ej).max() <= t * np.abs(ej).max()
    assert np.abs(vjp.cpu().numpy()[ks] - ev).max() <= t * np.abs(ev).max()
    ws = m.sr_prepare(to_dev(p), to_dev(s))
    got = m.sr_matvec(to_dev(s), ws, to_dev(v), diag_shift=0.01).cpu().numpy()
    exp = orbm.vjp_entries(pe, s, ej - ej.mean(), ks, N, M, rt) / n + 0.01 * v[ks]
    scale = np.abs(orbm.vjp_entries(pe, s, ej, ks, N, M, rt)).max() / n
    assert np.abs(got[ks] - exp).max() <= t * scale


@pytest.mark.parametrize("name,n", [("tfim100_cplx_f32_m32", 130), ("tfim150_cplx_f32_m100", 97),
                                    ("tfim300_real_f32", 70)])
def test_jacobian_products_many_sites(lib, name, n):
    """O v and O^dagger u where the sites span several staged windows of the FP32
    Jacobian-vector kernel (N above 64, 128 or 256 for one, two or four hidden chunks per
    block), on ragged sample counts; every entry against the oracle's explicit O."""
    m, om = cases.build(lib, name)
    N, M = om.n_sites, om.n_hidden
    p = cases.params(name, seed=85)
    pe = cases.oracle_params(name, p)
    s = cases.configs(name, n, seed=22)
    rng = np.random.default_rng(23)
    P = m.n_params
    u = rng.normal(size=n)
    v = rng.normal(size=P)
    if m.is_complex:
        u = u + 1j * rng.normal(size=n)
        v = v + 1j * rng.normal(size=P)
    vjp, jvp = m.log_psi_grad(to_dev(p), to_dev(s), u=to_dev(u), v=to_dev(v))
    O = orbm.log_derivatives(pe, s, N, M)
    if not m.is_complex:
        O = O.real
    ej = O @ v
    ev = O.conj().T @ u
    t = cases.tol(name)
    assert np.abs(jvp.cpu().numpy() - ej).max() <= t * np.abs(ej).max()
    assert np.abs(vjp.cpu().numpy() - ev).max() <= t * np.abs(ev).max()


def _jvp_rows(pe, s, v, N, M, rt, chunk=1024):
    """O v for many samples without forming O: (O v)_s = sum_i va_i s_i +
    sum_j t_sj (vb_j + sum_i vW_ji s_i), t = tanh theta (rounded by rt when given)."""
    va, vb, vW = v[:N], v[N:N + M], v[N + M:].reshape(M, N)
    out = []
    for i in range(0, len(s), chunk):
        sc = s[i:i + chunk].astype(np.float64)
        t = np.tanh(orbm.theta(pe, sc, N, M))
        if rt is not None:
            t = rt(t)
        out.append(sc @ va + np.sum(t * (vb[None, :] + sc @ vW.T), axis=1))
    return np.concatenate(out)


@pytest.mark.parametrize("name", NAMES)
def test_large_sv_and_vjp_at_workload_size(lib, name):
    """The 10x10 J1-J2 and 16x16 Heisenberg lattices at their workloads' 8192 samples per
    iteration (the same kernels, splits and reduction counts as the benchmark): every O v,
    and selected entries of O^dagger u and of S v, each from its own oracle column."""
    m, om = cases.build(lib, name)
    N, M = om.n_sites, om.n_hidden
    p = cases.params(name, theta=0.3, seed=87)
    pe = cases.oracle_params(name, p)
    rt = cases.round_tanh(name)
    n = 8192
    s = cases.configs(name, n, seed=24)
    rng = np.random.default_rng(25)
    P = m.n_params
    u = rng.normal(size=n) + 1j * rng.normal(size=n)
    v = rng.normal(size=P) + 1j * rng.normal(size=P)
    # the column-free product equals the oracle's O v on a few rows
    assert np.allclose(_jvp_rows(pe, s[:8], v, N, M, rt), orbm.jvp(pe, s[:8], v, N, M, rt),
                       rtol=1e-12, atol=1e-12)
    vjp, jvp = m.log_psi_grad(to_dev(p), to_dev(s), u=to_dev(u), v=to_dev(v))
    ej = _jvp_rows(pe, s, v, N, M, rt)
    ks = np.unique(np.concatenate([[0, N - 1, N, N + M - 1, N + M, P - 1],
                                   rng.integers(0, P, 40)]))
    ev = orbm.vjp_entries(pe, s, u, ks, N, M, rt)
    slack = 2e-3 if rt is not None else 0.0   # bfloat16 rounding ties of tanh(theta)
    t = cases.tol(name) + slack
    assert np.abs(jvp.cpu().numpy() - ej).max() <= t * np.abs(ej).max()
    assert np.abs(vjp.cpu().numpy()[ks] - ev).max() <= t * np.abs(ev).max()
    ws = m.sr_prepare(to_dev(p), to_dev(s))
    got = m.sr_matvec(to_dev(s), ws, to_dev(v), diag_shift=0.01).cpu().numpy()
    exp = orbm.vjp_entries(pe, s, ej - ej.mean(), ks, N, M, rt) / n + 0.01 * v[ks]
    scale = np.abs(orbm.vjp_entries(pe, s, ej, ks, N, M, rt)).max() / n
    assert np.abs(got[ks] - exp).max() <= t * scale
