"""Oracle: restricted-Boltzmann-machine wavefunction (test infrastructure only).

Sec. 2.2.2 of the paper: the RbmSpin machine is a fully complex RBM for spin-1/2
systems; an RBM is equivalent to a one-layer network with ln cosh activation (plus the
visible bias). Marginalising the M hidden units h_j in {+1,-1} of the RBM energy
a.sigma + sum_j h_j theta_j (the RBM of the paper's RBM reference) gives

    psi(sigma) = exp(a.sigma) * prod_j 2 cosh(theta_j),  theta_j = b_j + sum_i W_ji sigma_i.

We drop the constant M ln 2 (it cancels in every ratio and expectation), so

    log psi(sigma) = sum_i a_i sigma_i + sum_j ln cosh(theta_j).

Parameter packing (shared convention): p = [a (N) | b (M) | W (M x N, row j, column i)],
P = N + M + N*M entries, real or complex.

The log-derivatives O_k = d log psi / d p_k (Sec. 2.2.5: analytic for the RBM) are
O_a_i = sigma_i, O_b_j = tanh theta_j, O_W_ji = tanh(theta_j) sigma_i (holomorphic in p).

Pins (tests/test_oracle_rbm.py): log psi equals the brute-force sum over all 2**M hidden
configurations; special cases W=0 and a=b=0 (spin-flip symmetry); O_k equals central
finite differences of log psi.
"""
import numpy as np


def n_params(n_sites, n_hidden):
    return n_sites + n_hidden + n_sites * n_hidden


def unpack(params, n_sites, n_hidden):
    p = np.asarray(params)
    if p.shape != (n_params(n_sites, n_hidden),):
        raise ValueError("params has %s entries, expected %d" % (p.shape, n_params(n_sites, n_hidden)))
    a = p[:n_sites]
    b = p[n_sites:n_sites + n_hidden]
    W = p[n_sites + n_hidden:].reshape(n_hidden, n_sites)
    return a, b, W


def pack(a, b, W):
    return np.concatenate([np.ravel(a), np.ravel(b), np.ravel(W)])


def theta(params, sigma, n_sites, n_hidden):
    """theta[s, j] = b_j + sum_i W_ji sigma[s, i]  (sigma: [n, N])."""
    a, b, W = unpack(params, n_sites, n_hidden)
    s = np.asarray(sigma, dtype=np.float64)
    return b[None, :] + s @ W.T


def ln_cosh(z):
    """ln cosh z, computed without overflow as |Re z|-shifted form:
    ln cosh z = s z + log(1 + exp(-2 s z)) - ln 2 with s = sign(Re z).
    For complex z the imaginary part is only defined modulo 2 pi (and modulo pi when
    the sign choice flips); ratios exp(difference) are unaffected."""
    z = np.asarray(z)
    s = np.where(np.real(z) >= 0, 1.0, -1.0)
    return s * z + np.log1p(np.exp(-2.0 * s * z)) - np.log(2.0)


def log_psi(params, sigma, n_sites, n_hidden):
    """log psi for each row of sigma [n, N]."""
    a, b, W = unpack(params, n_sites, n_hidden)
    s = np.asarray(sigma, dtype=np.float64)
    th = theta(params, s, n_sites, n_hidden)
    return s @ a + ln_cosh(th).sum(axis=1)


def log_psi_hidden_sum(params, sigma, n_sites, n_hidden):
    """Definition by marginalisation over hidden units (exponential in M; pin only):
    log( sum_h exp(a.sigma + sum_j h_j theta_j) ) - M ln 2."""
    import itertools
    a, b, W = unpack(params, n_sites, n_hidden)
    s = np.asarray(sigma, dtype=np.float64)
    th = theta(params, s, n_sites, n_hidden)
    hs = np.array(list(itertools.product((1.0, -1.0), repeat=n_hidden)))   # [2^M, M]
    expo = (s @ a)[:, None] + th @ hs.T                                      # [n, 2^M]
    return np.log(np.exp(expo).sum(axis=1)) - n_hidden * np.log(2.0)


def log_derivatives(params, sigma, n_sites, n_hidden, round_tanh=None):
    """O[s, k] = d log psi(sigma_s) / d p_k, packed like p: [n, P]. round_tanh (optional)
    is applied to tanh(theta) first (the BF16 form's contractions read rounded rows)."""
    s = np.asarray(sigma, dtype=np.float64)
    th = theta(params, s, n_sites, n_hidden)
    t = np.tanh(th)
    if round_tanh is not None:
        t = round_tanh(t)
    n = s.shape[0]
    oW = t[:, :, None] * s[:, None, :]                    # [n, M, N], row j col i
    return np.concatenate([s.astype(t.dtype), t, oW.reshape(n, -1)], axis=1)


def jvp(params, sigma, v, n_sites, n_hidden, round_tanh=None):
    """(O v)_s = sum_k O_sk v_k  (no centering)."""
    return log_derivatives(params, sigma, n_sites, n_hidden, round_tanh) @ np.asarray(v)


def vjp(params, sigma, u, n_sites, n_hidden, round_tanh=None):
    """(O^dagger u)_k = sum_s conj(O_sk) u_s  (no centering, no 1/n)."""
    O = log_derivatives(params, sigma, n_sites, n_hidden, round_tanh)
    return O.conj().T @ np.asarray(u)


def vjp_entries(params, sigma, u, ks, n_sites, n_hidden, round_tanh=None):
    """Selected entries k of O^dagger u, each from its own column of O (for checks at
    sizes where the full [n, P] matrix does not fit): O[:, a_i] = sigma_i,
    O[:, b_j] = tanh(theta_j), O[:, W_ji] = tanh(theta_j) sigma_i."""
    a, b, W = unpack(params, n_sites, n_hidden)
    s = np.asarray(sigma, dtype=np.float64)
    u = np.asarray(u)
    out = []
    for k in ks:
        k = int(k)
        if k < n_sites:
            col = s[:, k]
        elif k < n_sites + n_hidden:
            j = k - n_sites
            col = np.tanh(b[j] + s @ W[j])
            if round_tanh is not None:
                col = round_tanh(col)
        else:
            j, i = divmod(k - n_sites - n_hidden, n_sites)
            t = np.tanh(b[j] + s @ W[j])
            if round_tanh is not None:
                t = round_tanh(t)
            col = t * s[:, i]
        out.append(np.sum(np.conj(col) * u))
    return np.array(out)
