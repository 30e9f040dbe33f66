"""Pins of the oracle RBM: hidden-unit marginalisation, special cases, finite differences."""
import numpy as np
import pytest

import synth
from oracle import rbm


@pytest.mark.parametrize("cplx", [False, True])
def test_log_psi_equals_hidden_sum(cplx):
    N, M = 6, 5
    p = synth.rbm_params(N, M, cplx, sigma=0.4, seed=3)
    s = synth.spin_configs(20, N, seed=4)
    a = rbm.log_psi(p, s, N, M)
    b = rbm.log_psi_hidden_sum(p, s, N, M)
    assert np.allclose(np.real(a), np.real(b), rtol=0, atol=1e-12)
    # imaginary parts agree modulo 2 pi
    d = np.imag(a) - np.imag(b)
    assert np.allclose(np.angle(np.exp(1j * d)), 0.0, atol=1e-12)


def test_special_cases():
    N, M = 7, 9
    p = synth.rbm_params(N, M, True, sigma=0.5, seed=5)
    a, b, W = rbm.unpack(p, N, M)
    s = synth.spin_configs(30, N, seed=6)
    p0 = rbm.pack(a, b, np.zeros_like(W))
    expect = s @ a + np.log(np.cosh(b)).sum()
    got = rbm.log_psi(p0, s, N, M)
    assert np.allclose(np.exp(got), np.exp(expect), rtol=1e-13)
    # a = b = 0: psi is even under global spin flip
    pz = rbm.pack(np.zeros_like(a), np.zeros_like(b), W)
    assert np.allclose(np.exp(rbm.log_psi(pz, s, N, M)), np.exp(rbm.log_psi(pz, -s, N, M)), rtol=1e-13)
    # large real theta: no overflow, ln cosh x ~ |x| - ln 2
    big = rbm.ln_cosh(np.array([800.0, -800.0]))
    assert np.allclose(big, 800.0 - np.log(2.0), rtol=1e-15)


@pytest.mark.parametrize("cplx", [False, True])
def test_log_derivatives_match_finite_differences(cplx):
    N, M = 5, 4
    p = synth.rbm_params(N, M, cplx, sigma=0.3, seed=8)
    s = synth.spin_configs(6, N, seed=9)
    O = rbm.log_derivatives(p, s, N, M)
    eps = 1e-6
    for k in range(p.size):
        dp = np.zeros_like(p)
        dp[k] = eps
        fd = (rbm.log_psi(p + dp, s, N, M) - rbm.log_psi(p - dp, s, N, M)) / (2 * eps)
        assert np.allclose(fd, O[:, k], rtol=1e-7, atol=1e-8), k


def test_jvp_vjp_adjoint():
    N, M = 6, 8
    p = synth.rbm_params(N, M, True, sigma=0.2, seed=10)
    s = synth.spin_configs(12, N, seed=11)
    v = synth.random_vector(p.size, True, 12)
    u = synth.random_vector(12, True, 13)
    lhs = np.vdot(u, rbm.jvp(p, s, v, N, M))
    rhs = np.vdot(rbm.vjp(p, s, u, N, M), v)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("rounded", [False, True])
def test_vjp_entries_equal_full_vjp(cplx, rounded):
    # every entry k of O^dagger u taken from its own column equals the full product; the
    # shapes have N != M so a swapped (row, column) index of W cannot pass
    from oracle import quant
    N, M = 5, 3
    p = synth.rbm_params(N, M, cplx, sigma=0.7, seed=21)
    s = synth.spin_configs(17, N, seed=22)
    u = synth.random_vector(17, cplx, 23)
    rt = quant.bf16 if rounded else None
    full = rbm.vjp(p, s, u, N, M, round_tanh=rt)
    ks = np.arange(p.size)
    got = rbm.vjp_entries(p, s, u, ks, N, M, round_tanh=rt)
    assert np.allclose(got, full, rtol=1e-13, atol=1e-13)
    # and the explicit O built element by element from the definition
    a, b, W = rbm.unpack(p, N, M)
    t_of = (lambda x: rt(x)) if rt is not None else (lambda x: x)
    for k in [0, N - 1, N, N + M - 1, N + M, N + M + 1, N + M + N, p.size - 1]:
        if k < N:
            col = s[:, k].astype(float)
        elif k < N + M:
            col = t_of(np.tanh(b[k - N] + s @ W[k - N]))
        else:
            j, i = (k - N - M) // N, (k - N - M) % N
            th = b[j] + sum(W[j, q] * s[:, q] for q in range(N))
            col = t_of(np.tanh(th)) * s[:, i]
        ref = np.sum(np.conj(col) * u)
        assert abs(got[k] - ref) < 1e-12 * max(1.0, abs(ref)), k
