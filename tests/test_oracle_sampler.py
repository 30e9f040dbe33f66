"""Pins of the oracle Metropolis sampler: one-step transition probabilities against the
analytic Metropolis kernel, and the stationary histogram against exact |psi|^2."""
import numpy as np
import pytest

import synth
from oracle import exact, lattice, rbm, sampler
from oracle.hamiltonian import HEISENBERG, MOVE_EXCHANGE, MOVE_FLIP, TFIM, Model


def model(move, n=6, m=4):
    b, sub = lattice.hypercube(n, 1)
    ham = TFIM if move == MOVE_FLIP else HEISENBERG
    return Model(n, m, b, ham=ham, J=(1.0, 0.0), h=1.0, sublattice=sub, move=move, is_complex=True)


@pytest.mark.parametrize("move", [MOVE_FLIP, MOVE_EXCHANGE])
def test_transition_row_matches_metropolis_kernel(move):
    m = model(move)
    N, M = m.n_sites, m.n_hidden
    p = synth.rbm_params(N, M, True, sigma=0.6, seed=31)
    s0 = np.array([1, -1, -1, 1, 1, -1], dtype=np.int8)
    trials = 40000
    sig = np.repeat(s0[None, :], trials, axis=0)
    ids = np.arange(trials, dtype=np.uint64)
    acc, _, _ = sampler.metropolis_step(m, p, sig, seed=77, chain_ids=ids, sweep=5, step=2)
    lp0 = rbm.log_psi(p, s0[None, :], N, M)[0]
    moves = []
    if move == MOVE_FLIP:
        for i in range(N):
            t = s0.copy(); t[i] = -t[i]; moves.append((t, 1.0 / N))
    else:
        B = m.bonds[0].shape[0]
        for i, k in m.bonds[0]:
            t = s0.copy(); t[i], t[k] = s0[k], s0[i]; moves.append((t, 1.0 / B))
    expect = {}
    for t, q in moves:
        if np.array_equal(t, s0):
            continue
        r = np.exp(2 * np.real(rbm.log_psi(p, t[None, :], N, M)[0] - lp0))
        expect[t.tobytes()] = expect.get(t.tobytes(), 0.0) + q * min(1.0, r)
    keys, counts = np.unique([row.tobytes() for row in sig], return_counts=True)
    got = dict(zip(keys, counts / trials))
    for k, pe in expect.items():
        pg = got.get(k, 0.0)
        assert abs(pg - pe) < 5 * np.sqrt(pe * (1 - pe) / trials) + 1e-4, (pg, pe)
    stay = 1.0 - sum(expect.values())
    assert abs(got.get(s0.tobytes(), 0.0) - stay) < 5 * np.sqrt(stay * (1 - stay) / trials) + 1e-4
    n_stay = int(np.sum(np.all(sig == s0[None, :], axis=1)))
    assert int(acc.sum()) == trials - n_stay


@pytest.mark.parametrize("move", [MOVE_FLIP, MOVE_EXCHANGE])
def test_stationary_histogram_chi_square(move):
    from scipy.stats import chi2
    m = model(move)
    N, M = m.n_sites, m.n_hidden
    p = synth.rbm_params(N, M, True, sigma=0.25, seed=33)  # one sweep damps the slowest mode by >= 7%
    chains = 3000
    init = sampler.init_chains(m, chains, seed=91)
    smp, last, nacc = sampler.sample(m, p, init, n_sweeps=1, n_discard=200, seed=91, counter=0)
    confs, pi = exact.exact_probabilities(m, p)
    if move == MOVE_EXCHANGE:
        keep = confs.sum(axis=1) == 0
        confs, pi = confs[keep], pi[keep] / pi[keep].sum()
    index = {c.tobytes(): k for k, c in enumerate(confs)}
    hist = np.zeros(len(confs))
    for row in last:
        hist[index[row.tobytes()]] += 1
    expct = pi * chains
    stat = np.sum((hist - expct) ** 2 / expct)
    pval = chi2.sf(stat, df=len(confs) - 1)
    assert pval > 1e-3, (stat, pval)


def test_init_chains():
    m = model(MOVE_EXCHANGE, n=10)
    c = sampler.init_chains(m, 500, seed=3)
    assert np.all(c.sum(axis=1) == 0)
    assert len({r.tobytes() for r in c}) > 200
    f = sampler.init_chains(model(MOVE_FLIP, n=10), 500, seed=3)
    assert abs(f.mean()) < 0.05


@pytest.mark.parametrize("move", [MOVE_FLIP, MOVE_EXCHANGE])
def test_init_chains_uniform_chi_square(move):
    # chain initialisation draws uniformly from every allowed configuration: all 2^6
    # spin rows (flip moves) or all 20 zero-magnetisation rows of six sites (a Fisher-
    # Yates shuffle whose swap partner is drawn from [0, k] for position k; drawing it
    # from [0, k) instead, Sattolo's cyclic shuffle, is not uniform here and fails)
    from scipy.stats import chi2
    m = model(move)
    chains = 24000
    c = sampler.init_chains(m, chains, seed=12)
    from oracle import lattice
    confs = lattice.all_configs(6)
    if move == MOVE_EXCHANGE:
        confs = confs[confs.sum(axis=1) == 0]
        assert len(confs) == 20
    index = {r.tobytes(): k for k, r in enumerate(confs)}
    hist = np.zeros(len(confs))
    for r in c:
        hist[index[r.tobytes()]] += 1
    expct = chains / len(confs)
    stat = np.sum((hist - expct) ** 2 / expct)
    assert chi2.sf(stat, df=len(confs) - 1) > 1e-3, stat


@pytest.mark.parametrize("move,cplx", [(MOVE_FLIP, False), (MOVE_FLIP, True), (MOVE_EXCHANGE, True),
                                       (MOVE_EXCHANGE, False)])
def test_cached_sampler_equals_definition(move, cplx):
    # the cached-angle chains equal the recompute-from-scratch chains on the same stream
    # (decisions could differ only at exact near-ties, none of which occur here)
    b, sub = lattice.hypercube(10, 1)
    ham = TFIM if move == MOVE_FLIP else HEISENBERG
    m = Model(10, 13, b, ham=ham, J=(1.0, 0.0), h=1.0, sublattice=sub, move=move, is_complex=cplx)
    p = synth.rbm_params(10, 13, cplx, sigma=0.4, seed=35)
    init = sampler.init_chains(m, 24, seed=36)
    a1, l1, n1 = sampler.sample(m, p, init, 6, 3, seed=36, counter=11)
    a2, l2, n2 = sampler.sample_cached(m, p, init, 6, 3, seed=36, counter=11)
    assert np.array_equal(a1, a2) and np.array_equal(l1, l2) and np.array_equal(n1, n2)
    assert n1.sum() > 0


def test_pt_with_one_replica_is_the_plain_sampler():
    m = model(MOVE_EXCHANGE, n=8)
    p = synth.rbm_params(8, 4, True, sigma=0.5, seed=40)
    init = sampler.init_chains(m, 12, seed=41)
    a, la, na = sampler.sample(m, p, init, 5, 2, seed=41, counter=3)
    b, lb, tb, ns = sampler.sample_pt(m, p, init[:, None, :], np.zeros((12, 1)), 5, 2, seed=41,
                                      counter=3)
    assert np.array_equal(a, b) and np.array_equal(la, lb[:, 0]) and ns.sum() == 0


@pytest.mark.parametrize("move", [MOVE_FLIP, MOVE_EXCHANGE])
def test_pt_samples_follow_psi_squared(move):
    # long tempered chains (3 replicas): the configurations recorded from the beta = 1
    # replica follow exact |psi|^2, and the temperatures are exchanged
    from scipy.stats import chi2
    m = model(move)
    N, M = m.n_sites, m.n_hidden
    p = synth.rbm_params(N, M, True, sigma=0.25, seed=43)
    chains, R = 1500, 3
    init = np.stack([sampler.init_chains(m, chains, seed=44 + r) for r in range(R)], axis=1)
    tix = np.tile(np.arange(R), (chains, 1))
    smp, _, tix2, nsw = sampler.sample_pt(m, p, init, tix, 1, 150, seed=44, counter=0)
    assert nsw.mean() > 10
    confs, pi = exact.exact_probabilities(m, p)
    if move == MOVE_EXCHANGE:
        keep = confs.sum(axis=1) == 0
        confs, pi = confs[keep], pi[keep] / pi[keep].sum()
    index = {c.tobytes(): k for k, c in enumerate(confs)}
    hist = np.zeros(len(confs))
    for row in smp.reshape(-1, N):
        hist[index[row.tobytes()]] += 1
    expct = pi * hist.sum()
    stat = np.sum((hist - expct) ** 2 / expct)
    assert chi2.sf(stat, df=len(confs) - 1) > 1e-3, stat


@pytest.mark.parametrize("move", [MOVE_FLIP, MOVE_EXCHANGE])
def test_pt_hot_replicas_follow_tempered_distribution(move):
    # after a long run the replica holding temperature index k is distributed as
    # |psi|^(2 beta_k) / Z (beta_k = 1 - k / R): a check of the beta weighting of both the
    # Metropolis and the exchange decisions, across independent chains
    from scipy.stats import chi2
    m = model(move)
    N, M = m.n_sites, m.n_hidden
    p = synth.rbm_params(N, M, True, sigma=0.4, seed=47)
    chains, R = 2000, 3
    init = np.stack([sampler.init_chains(m, chains, seed=48 + r) for r in range(R)], axis=1)
    tix = np.tile(np.arange(R), (chains, 1))
    _, last, tix2, _ = sampler.sample_pt(m, p, init, tix, 1, 120, seed=48, counter=0)
    confs, pi1 = exact.exact_probabilities(m, p)
    if move == MOVE_EXCHANGE:
        keep = confs.sum(axis=1) == 0
        confs, pi1 = confs[keep], pi1[keep]
    index = {c.tobytes(): k for k, c in enumerate(confs)}
    for k in (1, 2):
        beta = sampler.pt_betas(R)[k]
        pk = pi1 ** beta
        pk = pk / pk.sum()
        rows = last[np.arange(chains), np.argmax(tix2 == k, axis=1)]
        hist = np.zeros(len(confs))
        for row in rows:
            hist[index[row.tobytes()]] += 1
        stat = np.sum((hist - pk * chains) ** 2 / (pk * chains))
        assert chi2.sf(stat, df=len(confs) - 1) > 1e-3, (k, stat)
        # and not the beta = 1 distribution (the pin sees beta)
        p1 = pi1 / pi1.sum()
        stat1 = np.sum((hist - p1 * chains) ** 2 / (p1 * chains))
        assert chi2.sf(stat1, df=len(confs) - 1) < 1e-3, (k, stat1)
