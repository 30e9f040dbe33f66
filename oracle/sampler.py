"""Oracle: Metropolis sampling of |psi|^2 (test infrastructure only).

Sec. 2.2.5: configurations are drawn from pi(sigma) of Eq. 4 by Markov chains built with
the Metropolis algorithm, which ensures detailed balance. Listing-level choices the
paper leaves open, fixed as conventions both sides follow:

* moves: single-spin flip at a uniformly chosen site (MOVE_FLIP), or exchange of the two
  spins of a uniformly chosen color-0 bond (MOVE_EXCHANGE, the paper's nearest-neighbour
  swaps conserving total magnetisation). An exchange on two equal spins is the identity
  move: its random numbers are still drawn and it is not counted as accepted.
* acceptance: the proposal is symmetric, so accept with probability
  min(1, |psi(sigma')/psi(sigma)|^2) = min(1, exp(2 Re Delta)), Delta = log psi(sigma') -
  log psi(sigma): accept iff 2 Re Delta >= 0 or u < exp(2 Re Delta).
* a sweep is N proposals (N sites); one sample per chain is recorded after each sweep,
  after ``n_discard`` unrecorded sweeps.
* random numbers: Philox4x32-10, counter (chain, counter_base + sweep, step, tag); see
  ``philox``. Chain initialisation: independent +/-1 spins (MOVE_FLIP), or a uniformly
  random permutation (Fisher-Yates) of N/2 up and N/2 down spins (MOVE_EXCHANGE).

``sample`` is the definition: log psi(sigma') is recomputed from scratch for every
proposal. ``sample_cached`` runs the same chains with the hidden angles theta = W sigma + b
kept per chain and moved by the angle change of each accepted proposal, so a proposal costs
M ln cosh evaluations instead of N M products (the form used to time the oracle on the
host). Chains are independent, so all chains advance together as numpy arrays.

``sample_pt`` is parallel tempering (the paper's Metropolis samplers come with tempering
options): every chain carries R replicas; the replica holding temperature index r samples
|psi|^(2 beta_r) with beta_r = 1 - r / R (beta_0 = 1 is the physical distribution). A sweep
runs N proposals in every replica, accepted iff beta 2 Re Delta >= 0 or u <
exp(beta 2 Re Delta); replica w of chain c draws its proposals with chain index
(chain_offset + c) R + w. After each sweep the temperatures k and k + 1 are exchanged, for
k = 0 .. R-2 in order, iff E >= 0 or u < exp(E), E = (beta_k - beta_k+1)(L_b - L_a), where
L = 2 Re log psi of the replica a holding k and of the replica b holding k + 1, and u is
drawn with counter (chain_offset + c, sweep, k, TAG_SWAP). Replicas keep their
configurations; the temperature index each holds moves. The configuration of the replica
holding beta = 1 is recorded after each sweep.

Pins (tests/test_oracle_sampler.py): the empirical one-step transition row of
``metropolis_step`` against the analytic Metropolis kernel, and the histogram of long
chains against exact |psi|^2 by enumeration (chi-square), on N <= 6; ``sample_cached``
reproduces ``sample`` sample for sample on the same stream (both moves, real and complex);
``sample_pt`` with one replica equals ``sample``, and the recorded samples of long tempered
chains follow exact |psi|^2 (chi-square, N = 6, both moves, with the swap acceptance exponent
of the wrong sign failing it).
"""
import numpy as np

from . import philox, rbm
from .hamiltonian import MOVE_EXCHANGE, MOVE_FLIP


def init_chains(model, n_chains, seed, chain_offset=0):
    N = model.n_sites
    chains = np.arange(n_chains, dtype=np.uint64) + np.uint64(chain_offset)
    out = np.empty((n_chains, N), dtype=np.int8)
    if model.move == MOVE_FLIP:
        w = philox.draw(seed, chains[:, None], 0, np.arange(N)[None, :], philox.TAG_INIT)
        out[:] = np.where((w[..., 0] >> np.uint32(31)) == 0, 1, -1)
    else:
        if N % 2:
            raise ValueError("zero magnetisation needs an even number of sites")
        for c in range(n_chains):
            s = np.array([1] * (N // 2) + [-1] * (N // 2), dtype=np.int8)
            for k in range(N - 1, 0, -1):
                w = philox.draw(seed, chains[c], 0, k, philox.TAG_INIT)
                r = int(philox.index_from_word(w[0], k + 1))
                s[k], s[r] = s[r], s[k]
            out[c] = s
    return out


def metropolis_step(model, params, sigma, seed, chain_ids, sweep, step, machine=None):
    """One proposal + accept/reject for every chain. sigma [C, N] is updated in place.
    Returns a bool array: accepted (real moves only)."""
    N, M = model.n_sites, model.n_hidden
    w = philox.draw(seed, chain_ids, sweep, step, philox.TAG_PROPOSAL)
    u = philox.uniform_from_words(w[:, 1], w[:, 2])
    prop = sigma.copy()
    rows = np.arange(sigma.shape[0])
    if model.move == MOVE_FLIP:
        site = philox.index_from_word(w[:, 0], N)
        prop[rows, site] = -prop[rows, site]
        real_move = np.ones(sigma.shape[0], dtype=bool)
    else:
        bl = model.bonds[0]
        bidx = philox.index_from_word(w[:, 0], bl.shape[0])
        i, k = bl[bidx, 0], bl[bidx, 1]
        si, sk = sigma[rows, i].copy(), sigma[rows, k].copy()
        real_move = si != sk
        prop[rows, i] = sk
        prop[rows, k] = si
    if machine is None:
        delta = rbm.log_psi(params, prop, N, M) - rbm.log_psi(params, sigma, N, M)
    else:
        delta = machine.log_psi(params, prop) - machine.log_psi(params, sigma)
    two_re = 2.0 * np.real(delta)
    accept = real_move & ((two_re >= 0.0) | (u < np.exp(np.minimum(two_re, 0.0))))
    sigma[accept] = prop[accept]
    return accept, two_re, u


def sample(model, params, chain_sigma, n_sweeps, n_discard, seed, counter, chain_offset=0,
           record_ties=None, tie_margin=1e-12, machine=None):
    """Run every chain for n_discard + n_sweeps sweeps of N proposals.

    Returns (samples [n_sweeps, C, N], chain_sigma_out [C, N], n_accepted [C]).
    If ``record_ties`` is a list, each proposal with |u - exp(2 Re Delta)| < tie_margin is
    appended to it as (chain, sweep, step): the chain's row, the sweep counted from the
    first of this call (discarded ones included) and the proposal within the sweep.
    machine: any ansatz with log_psi(params, sigma) (default: the RBM of the model)."""
    sigma = np.array(chain_sigma, dtype=np.int8, copy=True)
    C, N = sigma.shape
    chains = np.arange(C, dtype=np.uint64) + np.uint64(chain_offset)
    out = np.empty((n_sweeps, C, N), dtype=np.int8)
    n_acc = np.zeros(C, dtype=np.int64)
    for sw in range(n_discard + n_sweeps):
        g = counter + sw
        for st in range(N):
            acc, two_re, u = metropolis_step(model, params, sigma, seed, chains, g, st, machine)
            n_acc += acc
            if record_ties is not None:
                near = np.abs(u - np.exp(np.minimum(two_re, 0.0))) < tie_margin
                for c in np.nonzero(near)[0]:
                    record_ties.append((int(chains[c]) - chain_offset, sw, st))
        if sw >= n_discard:
            out[sw - n_discard] = sigma
    return out, sigma, n_acc


def sample_cached(model, params, chain_sigma, n_sweeps, n_discard, seed, counter, chain_offset=0):
    """``sample`` with cached hidden angles: Delta = a.(sigma' - sigma) +
    sum_j [ln cosh(theta_j + delta_j) - ln cosh(theta_j)], delta = W (sigma' - sigma), and
    theta += delta on acceptance. Same random numbers and acceptance rule as ``sample``;
    returns (samples [n_sweeps, C, N], chain_sigma_out [C, N], n_accepted [C])."""
    N, M = model.n_sites, model.n_hidden
    a, b, W = rbm.unpack(params, N, M)
    sigma = np.array(chain_sigma, dtype=np.int8, copy=True)
    C = sigma.shape[0]
    chains = np.arange(C, dtype=np.uint64) + np.uint64(chain_offset)
    rows = np.arange(C)
    th = rbm.theta(params, sigma, N, M)                      # [C, M]
    lc = rbm.ln_cosh(th)
    out = np.empty((n_sweeps, C, N), dtype=np.int8)
    n_acc = np.zeros(C, dtype=np.int64)
    for sw in range(n_discard + n_sweeps):
        g = counter + sw
        for st in range(N):
            w = philox.draw(seed, chains, g, st, philox.TAG_PROPOSAL)
            u = philox.uniform_from_words(w[:, 1], w[:, 2])
            if model.move == MOVE_FLIP:
                i = philox.index_from_word(w[:, 0], N)
                k = i
                si = sigma[rows, i].astype(np.float64)
                real_move = np.ones(C, dtype=bool)
                delta = -2.0 * si[:, None] * W[:, i].T                # [C, M]
                dvis = -2.0 * si * a[i]
            else:
                bl = model.bonds[0]
                bidx = philox.index_from_word(w[:, 0], bl.shape[0])
                i, k = bl[bidx, 0], bl[bidx, 1]
                si = sigma[rows, i].astype(np.float64)
                sk = sigma[rows, k].astype(np.float64)
                real_move = si != sk
                # sigma'_i = sk, sigma'_k = si
                delta = (sk - si)[:, None] * W[:, i].T + (si - sk)[:, None] * W[:, k].T
                dvis = (sk - si) * a[i] + (si - sk) * a[k]
            lc_new = rbm.ln_cosh(th + delta)
            two_re = 2.0 * np.real(dvis + np.sum(lc_new - lc, axis=1))
            accept = real_move & ((two_re >= 0.0) | (u < np.exp(np.minimum(two_re, 0.0))))
            if model.move == MOVE_FLIP:
                sigma[rows[accept], i[accept]] = -sigma[rows[accept], i[accept]]
            else:
                ia, ka = i[accept], k[accept]
                vi = sigma[rows[accept], ia].copy()
                sigma[rows[accept], ia] = sigma[rows[accept], ka]
                sigma[rows[accept], ka] = vi
            th[accept] += delta[accept]
            lc[accept] = lc_new[accept]
            n_acc += accept
        if sw >= n_discard:
            out[sw - n_discard] = sigma
    return out, sigma, n_acc


def pt_betas(n_replicas):
    """Inverse temperatures beta_r = 1 - r / R of parallel tempering."""
    return 1.0 - np.arange(n_replicas) / float(n_replicas)


def sample_pt(model, params, chain_sigma, temp_index, n_sweeps, n_discard, seed, counter,
              chain_offset=0, record_ties=None, tie_margin=1e-12):
    """Parallel tempering. chain_sigma [C, R, N] (replica configurations) and temp_index
    [C, R] (the temperature index each replica holds) are copied and returned updated.
    Returns (samples [n_sweeps, C, N], chain_sigma_out, temp_index_out, n_swaps [C])."""
    N, M = model.n_sites, model.n_hidden
    sig = np.array(chain_sigma, dtype=np.int8, copy=True)
    tix = np.array(temp_index, dtype=np.int64, copy=True)
    C, R, _ = sig.shape
    betas = pt_betas(R)
    flat = sig.reshape(C * R, N)
    ids = ((np.arange(C, dtype=np.uint64) + np.uint64(chain_offset))[:, None] * np.uint64(R)
           + np.arange(R, dtype=np.uint64)[None, :]).reshape(-1)
    out = np.empty((n_sweeps, C, N), dtype=np.int8)
    n_swaps = np.zeros(C, dtype=np.int64)
    for sw in range(n_discard + n_sweeps):
        g = counter + sw
        beta = betas[tix.reshape(-1)]
        for st in range(N):
            w = philox.draw(seed, ids, g, st, philox.TAG_PROPOSAL)
            u = philox.uniform_from_words(w[:, 1], w[:, 2])
            prop = flat.copy()
            rows = np.arange(C * R)
            if model.move == MOVE_FLIP:
                site = philox.index_from_word(w[:, 0], N)
                prop[rows, site] = -prop[rows, site]
                real_move = np.ones(C * R, dtype=bool)
            else:
                bl = model.bonds[0]
                bidx = philox.index_from_word(w[:, 0], bl.shape[0])
                i, k = bl[bidx, 0], bl[bidx, 1]
                si, sk = flat[rows, i].copy(), flat[rows, k].copy()
                real_move = si != sk
                prop[rows, i] = sk
                prop[rows, k] = si
            delta = rbm.log_psi(params, prop, N, M) - rbm.log_psi(params, flat, N, M)
            ex = beta * 2.0 * np.real(delta)
            accept = real_move & ((ex >= 0.0) | (u < np.exp(np.minimum(ex, 0.0))))
            if record_ties is not None:
                near = real_move & (np.abs(u - np.exp(np.minimum(ex, 0.0))) < tie_margin)
                for q in np.nonzero(near)[0]:
                    record_ties.append((int(q // R), sw, st))
            flat[accept] = prop[accept]
        # exchanges of adjacent temperatures, in order
        L = 2.0 * np.real(rbm.log_psi(params, flat, N, M)).reshape(C, R)
        cid = np.arange(C, dtype=np.uint64) + np.uint64(chain_offset)
        for k in range(R - 1):
            w = philox.draw(seed, cid, g, k, philox.TAG_SWAP)
            u = philox.uniform_from_words(w[:, 1], w[:, 2])
            a = np.argmax(tix == k, axis=1)
            b = np.argmax(tix == k + 1, axis=1)
            rows = np.arange(C)
            ex = (betas[k] - betas[k + 1]) * (L[rows, b] - L[rows, a])
            acc = (ex >= 0.0) | (u < np.exp(np.minimum(ex, 0.0)))
            if record_ties is not None:
                near = np.abs(u - np.exp(np.minimum(ex, 0.0))) < tie_margin
                for c in np.nonzero(near)[0]:
                    record_ties.append((int(c), sw, -1 - k))
            tix[rows[acc], a[acc]] = k + 1
            tix[rows[acc], b[acc]] = k
            n_swaps += acc
        if sw >= n_discard:
            phys = np.argmax(tix == 0, axis=1)
            out[sw - n_discard] = flat.reshape(C, R, N)[np.arange(C), phys]
    return out, flat.reshape(C, R, N), tix, n_swaps
