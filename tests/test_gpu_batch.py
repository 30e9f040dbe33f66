"""GPU parity of batches of independent models (uneven sizes) sampled in one launch:
every model's chains, samples and local energies against the oracle run on that model
alone with the model's seed (seed ^ k), and against the single-model entry points."""
import numpy as np
import pytest
import torch

import cases
import synth
from oracle import hamiltonian as oh, lattice as ol, sampler as osamp

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def make(lib, kinds, prec, cplx):
    """kinds: list of (kind, L, ndim, diag, h or J2, alpha)."""
    specs, oracles = [], []
    for kind, L, ndim, diag, c, alpha in kinds:
        bonds, sub = lib.nqs_hypercube(L, ndim, diag)
        ob, osub = ol.hypercube(L, ndim, with_diagonals=diag)
        N = L ** ndim
        if kind == "tfim":
            kw = dict(ham=lib.TFIM, J=(1.0, 0.0), h=c, marshall=False, move=lib.MOVE_FLIP)
            okw = dict(ham=oh.TFIM, J=(1.0, 0.0), h=c, marshall=False, move=oh.MOVE_FLIP)
        else:
            kw = dict(ham=lib.HEISENBERG, J=(1.0, c), h=0.0, marshall=True, move=lib.MOVE_EXCHANGE)
            okw = dict(ham=oh.HEISENBERG, J=(1.0, c), h=0.0, marshall=True, move=oh.MOVE_EXCHANGE)
        specs.append(dict(n_sites=N, n_hidden=alpha * N, bonds=bonds, sublattice=sub,
                          is_complex=cplx, prec=prec, **kw))
        oracles.append(oh.Model(N, alpha * N, ob, sublattice=osub, is_complex=cplx, **okw))
    return lib.Batch(specs), specs, oracles


def params_of(oracles, cplx, prec, seed):
    ps = []
    for k, om in enumerate(oracles):
        p = synth.rbm_params(om.n_sites, om.n_hidden, cplx, sigma=0.3 / np.sqrt(om.n_sites + 1.0)
                             if cplx else 1.5 / np.sqrt(om.n_sites + 1.0), seed=seed + k)
        if prec != 0:
            p = p.astype(np.complex64 if cplx else np.float32)
        ps.append(p)
    return ps


def check_batch(lib, kinds, prec, cplx, n_chains, margin, tol):
    b, specs, oracles = make(lib, kinds, prec, cplx)
    ps = params_of(oracles, cplx, prec, seed=100)
    params = to_dev(np.concatenate(ps))
    Ns = [om.n_sites for om in oracles]
    chains = torch.empty(sum(c * n for c, n in zip(n_chains, Ns)), dtype=torch.int8, device=DEV)
    b.chain_init(chains, n_chains, seed=9)
    init = chains.cpu().numpy().copy()
    S, D = 3, 2
    nacc = torch.zeros(sum(n_chains), dtype=torch.int64, device=DEV)
    smp, el = b.sample(params, chains, n_chains, S, D, seed=9, counter=5, n_accepted=nacc)
    smp, el, init_off = smp.cpu().numpy(), el.cpu().numpy(), 0
    so = eo = 0
    for k, om in enumerate(oracles):
        C, N = n_chains[k], om.n_sites
        pe = ps[k].astype(np.complex128 if cplx else np.float64)
        ini = init[init_off:init_off + C * N].reshape(C, N)
        assert np.array_equal(ini, osamp.init_chains(om, C, seed=9 ^ k)), k
        ties = []
        exp, _, _ = osamp.sample(om, pe, ini, S, D, seed=9 ^ k, counter=5, record_ties=ties,
                                 tie_margin=margin)
        got = smp[so:so + S * C * N].reshape(S, C, N)
        cases.compare_chains(got, exp, ties, D)
        eg = el[eo:eo + S * C]
        ee = oh.local_energy(om, pe, got.reshape(-1, N))
        assert np.abs(eg - ee).max() <= tol * max(1.0, np.abs(ee).max()), k
        # the single-model entry point with the model's seed gives the same chains
        m = lib.Model(**specs[k])
        ch1 = to_dev(ini.copy())
        s1, _ = m.sample(to_dev(ps[k]), ch1, S, D, seed=9 ^ k, counter=5)
        assert np.array_equal(s1.cpu().numpy(), got), k
        init_off += C * N
        so += S * C * N
        eo += S * C


def test_batch_tfim_uneven_fp32(lib):
    """Transverse-field Ising rings of 16 to 128 sites, alpha = 2, real FP32."""
    kinds = [("tfim", L, 1, False, h, 2) for L, h in
             [(16, 0.6), (23, 1.4), (40, 1.0), (64, 0.8), (100, 1.2), (128, 0.5)]]
    check_batch(lib, kinds, 1, False, [24, 7, 33, 16, 9, 12], 1e-4, 1e-5)


def test_batch_mixed_models_fp64(lib):
    """A TFIM ring, a Heisenberg ring and a 4x4 J1-J2 lattice, complex FP64."""
    kinds = [("tfim", 10, 1, False, 1.0, 1), ("heis", 12, 1, False, 0.0, 3),
             ("heis", 4, 2, True, 0.5, 4)]
    check_batch(lib, kinds, 0, True, [5, 17, 8], 1e-12, 1e-10)


def check_batch_sr(lib, kinds, prec, cplx, n_list, fp64):
    from oracle import rbm as orbm, sr as osr
    b, specs, oracles = make(lib, kinds, prec, cplx)
    ps = params_of(oracles, cplx, prec, seed=200)
    ss, els = [], []
    for k, om in enumerate(oracles):
        s = synth.spin_configs(n_list[k], om.n_sites, 300 + k,
                               zero_magnetisation=(om.move == oh.MOVE_EXCHANGE))
        pe = ps[k].astype(np.complex128 if cplx else np.float64)
        ss.append(s)
        els.append(oh.local_energy(om, pe, s))
    pt = to_dev(np.concatenate(ps))
    infos = b.sr_step(pt, to_dev(np.concatenate([s.reshape(-1) for s in ss])),
                      to_dev(np.concatenate(els)), n_list, lr=0.05, diag_shift=0.01, cg_tol=0.0,
                      cg_maxiter=12)
    got = pt.cpu().numpy()
    off = 0
    for k, om in enumerate(oracles):
        P = b.n_params[k]
        pe = ps[k].astype(np.complex128 if cplx else np.float64)
        p_new, io = osr.sr_step(om, pe, ss[k], els[k], lr=0.05, diag_shift=0.01, cg_tol=0.0,
                                cg_maxiter=12)
        assert infos[k]["cg_iters"] == io["iters"] == 12
        assert abs(infos[k]["energy_re"] - np.real(io["energy"])) <= 1e-10 * max(1, abs(io["energy"]))
        step_o = p_new - pe
        step_g = got[off:off + P].astype(pe.dtype) - pe
        if fp64:
            O = orbm.log_derivatives(pe, ss[k], om.n_sites, om.n_hidden)
            if not cplx:
                O = O.real
            tol = max(1e-9, 10 * cases.cg_sensitivity(O, els[k], 0.01, 12))
            assert np.abs(step_g - step_o).max() <= tol * np.abs(step_o).max(), k
        else:
            assert np.abs(step_g - step_o).max() <= 1e-4 * np.abs(step_o).max() + 1e-7, k
        off += P


def test_batch_sr_mixed_models_fp64(lib):
    kinds = [("tfim", 10, 1, False, 1.0, 1), ("heis", 12, 1, False, 0.0, 3),
             ("heis", 4, 2, True, 0.5, 4)]
    check_batch_sr(lib, kinds, 0, True, [300, 411, 257], True)


def test_batch_sr_tfim_uneven_fp32(lib):
    kinds = [("tfim", L, 1, False, h, 2) for L, h in [(16, 0.6), (23, 1.4), (40, 1.0), (64, 0.8)]]
    check_batch_sr(lib, kinds, 1, False, [512, 300, 640, 257], False)
