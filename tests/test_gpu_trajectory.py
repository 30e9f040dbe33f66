"""Whole-loop checks of variational Monte Carlo on the GPU (Sec. 2.2.5): a multi-step SR
trajectory against the oracle run on the same counter-based random stream, and
convergence of the GPU loop to exact ground energies (the 10-site transverse-field Ising
ring, and the 20-site Heisenberg ring of the paper's worked example, Fig. 2)."""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import hamiltonian as oh, lattice as ol, rbm as orbm, sampler as osamp, sr as osr

pytestmark = pytest.mark.gpu

DEV = "cuda"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "reference_energies.txt")


def golden(name):
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#") and line.split()[0] == name:
            return float(line.split()[1])
    raise KeyError(name)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def tfim10(lib, prec=0):
    bonds, sub = lib.nqs_hypercube(10, 1)
    m = lib.Model(10, 10, bonds, ham=lib.TFIM, J=(1.0, 0.0), h=1.0, sublattice=sub,
                  move=lib.MOVE_FLIP, is_complex=False, prec=prec)
    ob, osub = ol.hypercube(10, 1)
    om = oh.Model(10, 10, ob, ham=oh.TFIM, J=(1.0, 0.0), h=1.0, sublattice=osub,
                  move=oh.MOVE_FLIP, is_complex=False)
    return m, om


def test_sr_trajectory_matches_oracle(lib):
    """The 10-site TFIM ring, real FP64, alpha = 1, 16 chains: ten iterations of (sample 100
    sweeps, local energies, SR step), GPU and oracle each on their own state. Samples are
    bit-exact at every iteration (a chain may leave only after a recorded near-tie), the
    energies agree to 1e-10 and the parameters to 1e-9 relative of the step."""
    m, om = tfim10(lib)
    C, S, iters = 16, 100, 10
    p0 = synth.rbm_params(10, 10, False, sigma=0.01, seed=1234)
    ch = torch.empty((C, 10), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=1234)
    ch_o = osamp.init_chains(om, C, seed=1234)
    assert np.array_equal(ch.cpu().numpy(), ch_o)
    pg, po = to_dev(p0.copy()), p0.copy()
    counter = 0
    for it in range(iters):
        discard = 10 if it == 0 else 0
        smp, el = m.sample(pg, ch, S, discard, seed=1234, counter=counter, with_eloc=True)
        ties = []
        smp_o, ch_o, _ = osamp.sample(om, po, ch_o, S, discard, seed=1234, counter=counter,
                                      record_ties=ties, tie_margin=1e-12)
        counter += S + discard
        got = smp.cpu().numpy()
        assert not ties and np.array_equal(got, smp_o), it
        el_o = oh.local_energy(om, po, smp_o.reshape(-1, 10))
        assert np.abs(el.cpu().numpy() - el_o).max() <= 1e-10 * np.abs(el_o).max()
        info = m.sr_step(pg, smp.view(S * C, 10), el, lr=0.05, diag_shift=0.01, cg_tol=1e-10,
                         cg_maxiter=500, n_chains=C)
        p_new, io = osr.sr_step(om, po, smp_o.reshape(-1, 10), el_o, lr=0.05, diag_shift=0.01,
                                cg_tol=1e-10, cg_maxiter=500)
        mean, var, err = osr.stats(el_o, n_chains=C)
        assert abs(info["energy_re"] - mean) <= 1e-10 * abs(mean)
        assert abs(info["energy_err"] - err) <= 1e-8 * err
        step = np.abs(p_new - po).max()
        assert np.abs(pg.cpu().numpy() - p_new).max() <= 1e-9 * step, it
        po = p_new


def _run_vmc(lib, m, C, S, iters, lr, shift, seed, prec_dtype, complex_, P_sigma=0.01,
             cg_tol=1e-8, cg_maxiter=1000):
    """Plain VMC loop on the GPU; returns per-iteration (energy, error bar)."""
    p = synth.rbm_params(m.n_sites, m.n_hidden, complex_, sigma=P_sigma, seed=seed)
    pt = to_dev(p.astype(prec_dtype))
    ch = torch.empty((C, m.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=seed)
    smp = torch.empty((S, C, m.n_sites), dtype=torch.int8, device=DEV)
    el = torch.empty(S * C, dtype=m.value_dtype, device=DEV)
    ws = torch.empty(m.sr_workspace_bytes(S * C), dtype=torch.uint8, device=DEV)
    out = []
    counter = 0
    for it in range(iters):
        discard = 50 if it == 0 else 0
        m.sample(pt, ch, S, discard, seed=seed, counter=counter, samples=smp, eloc=el)
        counter += S + discard
        info = m.sr_step(pt, smp.view(S * C, m.n_sites), el, lr=lr, diag_shift=shift,
                         cg_tol=cg_tol, cg_maxiter=cg_maxiter, workspace=ws, n_chains=C)
        out.append((info["energy_re"], info["energy_err"], info["variance"]))
    return np.array(out)


def test_tfim10_vmc_converges_to_exact_energy(lib):
    """The 10-site TFIM ring (J = h = 1), real FP64 RBM with alpha = 1, 16 chains x 1000
    sweeps per iteration, SR shift 0.01. At lr 0.01 the 100 iterations of that workload
    reach an imaginary time of 1 only (the oracle's exact-expectation SR is still 6e-3
    above the ground energy there), so the loop runs 300 iterations at lr 0.05; the mean of
    the last 50 energies must lie within 3 of its error bars (plus the variational gap of
    the ansatz, 1e-4 relative, measured with the oracle's exact SR) of the closed form."""
    m, _ = tfim10(lib)
    e0 = golden("tfim_n10_h1")
    res = _run_vmc(lib, m, C=16, S=1000, iters=300, lr=0.05, shift=0.01, seed=1234,
                   prec_dtype=np.float64, complex_=False)
    tail = res[-50:]
    emean = tail[:, 0].mean()
    err = np.sqrt(np.mean(tail[:, 1] ** 2) / len(tail))
    print("TFIM10 VMC: E = %.8f +- %.2e (exact %.8f), variance %.3e"
          % (emean, err, e0, tail[:, 2].mean()))
    assert emean >= e0 - 3 * err - 1e-9
    assert emean - e0 <= 3 * err + 1e-4 * abs(e0)


def test_heisenberg20_vmc_paper_example(lib):
    """The paper's worked example (Sec. 2.2.5, Fig. 2): the 20-site Heisenberg ring,
    complex RBM with 20 hidden units (initial sigma 0.01, seed 1234), Marshall sign,
    exchange moves, SR. With the SR step read as p <- p - lr x (lr the imaginary-time
    step), the paper's lr 0.01 over 200 iterations is an imaginary time of 2 only: 1000
    samples per iteration then reach a relative error of a few 1e-3 (measured 3.4e-3), not
    the 4.16e-5 the paper reports at iteration 200. A longer run (lr 0.05, shift 0.001,
    10^4 samples, 600 iterations) reaches about 1.1e-4, where this ansatz (alpha = 1, no
    symmetry) levels off. Means of the last 20 iterations are compared."""
    bonds, sub = lib.nqs_hypercube(20, 1)
    m = lib.Model(20, 20, bonds, ham=lib.HEISENBERG, J=(1.0, 0.0), marshall=True,
                  sublattice=sub, move=lib.MOVE_EXCHANGE, is_complex=True, prec=lib.F64)
    e0 = golden("heis_ring_n20")
    res = _run_vmc(lib, m, C=100, S=10, iters=200, lr=0.01, shift=0.01, seed=1234,
                   prec_dtype=np.complex128, complex_=True)
    rel = np.abs(res[:, 0] - e0) / abs(e0)
    r200 = rel[-20:].mean()
    print("Heisenberg20 VMC, paper settings: rel. error %.3e at 200 iterations" % r200)
    assert rel[:20].mean() > 10 * r200 and r200 <= 6e-3
    assert np.all(res[:, 0] >= e0 - 5 * res[:, 1] - 1e-9)    # variational within noise
    res = _run_vmc(lib, m, C=1000, S=10, iters=600, lr=0.05, shift=0.001, seed=1234,
                   prec_dtype=np.complex128, complex_=True)
    r600 = abs(res[-20:, 0].mean() - e0) / abs(e0)
    print("Heisenberg20 VMC, 600 iterations at lr 0.05: rel. error %.3e" % r600)
    assert r600 <= 2e-4
