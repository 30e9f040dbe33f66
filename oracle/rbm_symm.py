"""Oracle: the symmetric RBM, RbmSpinSymm (test infrastructure only).

Sec. 2.2.2 of the paper lists, next to the plain RBM, an RBM whose weights respect the
symmetries of the lattice. With a group of G site permutations (g maps site i to
perm[g][i]; (T_g sigma)_i = sigma_perm[g][i]) and alpha filters, the hidden units are
labelled (f, g), f < alpha, g < G, and

    theta_fg(sigma) = b_f + sum_i W_fi sigma_perm[g][i],
    log psi(sigma)  = a sum_i sigma_i + sum_f sum_g ln cosh theta_fg(sigma)

(one visible bias a, one hidden bias b_f and one filter W_f. per filter; the constant of
2 cosh is dropped as for the RBM). Parameter packing: p = [a (1) | b (alpha) | W (alpha x N,
row f, column i)], P = 1 + alpha + alpha N.

Log-derivatives from the definition: O_a = sum_i sigma_i, O_bf = sum_g tanh theta_fg,
O_Wfi = sum_g tanh(theta_fg) sigma_perm[g][i].

``expand`` writes the same amplitude as a plain RBM with M = alpha G hidden units (unit
j = f G + g): b_j = b_f, a_i = a, and W_j,perm[g][i] = W_fi; it is used only to evaluate
local energies with the RBM oracle.

Pins (tests/test_oracle_rbm_symm.py): psi(T_h sigma) = psi(sigma) for every symmetry h;
log psi equals the brute-force sum over all 2^(alpha G) hidden configurations; the expanded
RBM gives the same log psi; O_k against central finite differences; translations of the
hypercube form a group (closure, identity).
"""
import itertools

import numpy as np

from . import rbm


def n_params(n_sites, alpha):
    return 1 + alpha + alpha * n_sites


def unpack(params, n_sites, alpha):
    p = np.asarray(params)
    if p.shape != (n_params(n_sites, alpha),):
        raise ValueError("params has %s entries, expected %d" % (p.shape, n_params(n_sites, alpha)))
    return p[0], p[1:1 + alpha], p[1 + alpha:].reshape(alpha, n_sites)


def translations(L, ndim):
    """The L^ndim translations of the periodic hypercube as site permutations: perm[g][i]
    is site i moved by the vector of g (site s = x0 + L x1, as in lattice.hypercube)."""
    n = L ** ndim
    perm = np.empty((n, n), dtype=np.int64)
    for g in range(n):
        gx, gy = g % L, (g // L if ndim == 2 else 0)
        for s in range(n):
            x, y = s % L, (s // L if ndim == 2 else 0)
            perm[g, s] = (x + gx) % L + (L * ((y + gy) % L) if ndim == 2 else 0)
    return perm


def theta(params, sigma, n_sites, alpha, perm):
    """theta[s, f, g] = b_f + sum_i W_fi sigma[s, perm[g][i]]."""
    a, b, W = unpack(params, n_sites, alpha)
    s = np.asarray(sigma, dtype=np.float64)
    sg = s[:, np.asarray(perm)]                      # [n, G, N]: sigma_perm[g][i]
    return b[None, :, None] + np.einsum("fi,ngi->nfg", W, sg)


def log_psi(params, sigma, n_sites, alpha, perm):
    a, b, W = unpack(params, n_sites, alpha)
    s = np.asarray(sigma, dtype=np.float64)
    th = theta(params, s, n_sites, alpha, perm)
    return a * s.sum(axis=1) + rbm.ln_cosh(th).sum(axis=(1, 2))


def log_psi_hidden_sum(params, sigma, n_sites, alpha, perm):
    """Marginalisation over all 2^(alpha G) hidden configurations (pin only)."""
    a, b, W = unpack(params, n_sites, alpha)
    s = np.asarray(sigma, dtype=np.float64)
    th = theta(params, s, n_sites, alpha, perm).reshape(s.shape[0], -1)
    K = th.shape[1]
    hs = np.array(list(itertools.product((1.0, -1.0), repeat=K)))
    expo = (a * s.sum(axis=1))[:, None] + th @ hs.T
    return np.log(np.exp(expo).sum(axis=1)) - K * np.log(2.0)


def log_derivatives(params, sigma, n_sites, alpha, perm):
    """O[s, k] = d log psi(sigma_s) / d p_k: [n, P]."""
    s = np.asarray(sigma, dtype=np.float64)
    t = np.tanh(theta(params, s, n_sites, alpha, perm))            # [n, alpha, G]
    sg = s[:, np.asarray(perm)]                                    # [n, G, N]
    oa = s.sum(axis=1, keepdims=True).astype(t.dtype)
    ob = t.sum(axis=2)
    oW = np.einsum("nfg,ngi->nfi", t, sg).reshape(s.shape[0], -1)
    return np.concatenate([oa, ob, oW], axis=1)


def expand(params, n_sites, alpha, perm):
    """Parameters of the plain RBM (M = alpha G) with the same amplitude."""
    a, b, W = unpack(params, n_sites, alpha)
    perm = np.asarray(perm)
    G = perm.shape[0]
    M = alpha * G
    dt = np.result_type(np.asarray(params).dtype, np.float64)
    ae = np.full(n_sites, a, dtype=dt)
    be = np.repeat(b, G).astype(dt)
    We = np.zeros((M, n_sites), dtype=dt)
    for f in range(alpha):
        for g in range(G):
            We[f * G + g, perm[g]] = W[f]
    return rbm.pack(ae, be, We)
