"""Complex FP32 parity at the |theta| of trained models (|theta| ~ 1 to 1.5, with hidden
angles near the poles of tanh), against the FP64 oracle, with per-entry tolerances
derived from the float rounding of theta (tests/fp32_bounds.py) instead of a fixed
relative tolerance: local energies, O v, entries of O^dagger u and of S v."""
import numpy as np
import pytest
import torch

import cases
import fp32_bounds as fb
from oracle import hamiltonian as oh, rbm as orbm

pytestmark = pytest.mark.gpu

DEV = "cuda"
NAMES = ["heis40_cplx_f32", "j1j2_4x4_cplx_f32", "tfim37_cplx_f32_m37", "heis6x6_cplx_f32"]


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("theta", [1.0, 1.5])
def test_fp32_local_energy_trained_scale(lib, name, theta):
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=theta, seed=301)
    pe = p.astype(np.complex128)
    s = cases.configs(name, 160, seed=302)
    got = m.local_energy(to_dev(p), to_dev(s)).cpu().numpy()
    exp = oh.local_energy(om, pe, s)
    bound = fb.local_energy_bound(om, pe, s)
    scale = np.abs(exp).max()
    err = np.abs(got - exp)
    # 2x the first-order bound, plus a floor far below the fixed 1e-5 relative tolerance
    assert np.all(err <= 2 * bound + 1e-7 * scale), (err / (bound + 1e-300)).max()
    # the regime is exercised: some samples' bounds exceed the fixed FP32 tolerance
    print("%s theta %.1f: max bound / (1e-5 |E|) = %.2f, max err / bound = %.3f"
          % (name, theta, (bound / (1e-5 * scale)).max(), (err / bound).max()))


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("theta", [1.0, 1.5])
def test_fp32_jacobian_and_sv_trained_scale(lib, name, theta):
    m, om = cases.build(lib, name)
    N, M = om.n_sites, om.n_hidden
    p = cases.params(name, theta=theta, seed=303)
    pe = p.astype(np.complex128)
    n = 333
    s = cases.configs(name, n, seed=304)
    rng = np.random.default_rng(305)
    P = m.n_params
    u = rng.normal(size=n) + 1j * rng.normal(size=n)
    v = rng.normal(size=P) + 1j * rng.normal(size=P)
    vjp, jvp = m.log_psi_grad(to_dev(p), to_dev(s), u=to_dev(u), v=to_dev(v))
    O = orbm.log_derivatives(pe, s, N, M)
    ej, ev = O @ v, O.conj().T @ u
    bj = fb.jvp_bound(pe, s, v, N, M)
    ks = np.arange(P)
    bv = fb.vjp_entries_bound(pe, s, u, ks, N, M)
    fl = 1e-7
    assert np.all(np.abs(jvp.cpu().numpy() - ej) <= 2 * bj + fl * np.abs(ej).max())
    assert np.all(np.abs(vjp.cpu().numpy() - ev) <= 2 * bv + fl * np.abs(ev).max())
    # S v: O^dagger of the centred y = O v, over n, and the shift
    ws = m.sr_prepare(to_dev(p), to_dev(s))
    got = m.sr_matvec(to_dev(s), ws, to_dev(v), diag_shift=0.01).cpu().numpy()
    yc = ej - ej.mean()
    exp = O.conj().T @ yc / n + 0.01 * v
    t = np.abs(np.tanh(orbm.theta(pe, s, N, M)))
    # the JVP error enters through every sample's y (and its mean): |O_sk| (|dy_s| + mean)
    dy = bj + bj.mean()
    colsum = np.concatenate([np.full(N, dy.sum()), (t * dy[:, None]).sum(axis=0),
                             np.repeat((t * dy[:, None]).sum(axis=0), N)])
    bs = (fb.vjp_entries_bound(pe, s, yc, ks, N, M) + colsum) / n
    assert np.all(np.abs(got - exp) <= 2 * bs + fl * np.abs(exp).max())
