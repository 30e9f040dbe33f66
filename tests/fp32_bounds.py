"""Rounding bounds of the FP32 form at any |theta| (test helper, float64 numpy).

In the FP32 form the Jacobian contractions and the local energies from rows read
t = tanh(theta) computed in float: theta_j = b_j + sum_i W_ji sigma_i is accumulated in
float (products with sigma = +/-1 are exact), so |d theta_j| <= gamma_{N+1} (|b_j| +
sum_i |W_ji|) with gamma_n = n u / (1 - n u), u = 2^-24 (the standard bound of recursive
summation, valid for any order). The float tanh then rounds its argument and its result;
its error is bounded by |sech^2 theta| (|d theta| + 4 u max(1, |theta|)) + 4 u (1 + |t|).
Near the poles of tanh (Im theta = pi/2) sech^2 grows without bound: these bounds give
the tolerance per sample there instead of avoiding that regime.

From the bound on t follow first-order bounds of the local energy (Eq. 5 through the
product form of the amplitude ratio), of O v, of entries of O^dagger u and of S v.
"""
import numpy as np

U32 = 2.0 ** -24


def gamma(n):
    return n * U32 / (1.0 - n * U32)


def unpack(p, N, M):
    return p[:N], p[N:N + M], p[N + M:].reshape(M, N)


def tanh_bounds(p, s, N, M):
    """theta [n, M], t = tanh theta [n, M] (float64) and the bound dt [n, M] of the float
    t the kernels use."""
    a, b, W = unpack(np.asarray(p), N, M)
    s = np.asarray(s, dtype=np.float64)
    th = b[None, :] + s @ W.T
    t = np.tanh(th)
    dth = gamma(N + 1) * (np.abs(b) + np.abs(W).sum(axis=1))[None, :]
    sech2 = np.abs(1.0 - t * t)
    dt = sech2 * (dth + 4 * U32 * np.maximum(1.0, np.abs(th))) + 4 * U32 * (1.0 + np.abs(t))
    return th, t, dt


def local_energy_bound(om, p, s):
    """Bound of |E_loc(float) - E_loc(exact)| per sample: every connected configuration c
    contributes |H_c r_c| (sum_j (|S_cj| dt_j + 4 u (|C_cj| + |t_j S_cj|)) / |term_cj| +
    2 M u), with term_cj = C_cj + t_j S_cj the factor of hidden unit j in the ratio r_c
    (C = cosh, S = sinh of the angle change, themselves rounded to float)."""
    from oracle import hamiltonian as oh
    N, M = om.n_sites, om.n_hidden
    a, b, W = unpack(np.asarray(p), N, M)
    th, t, dt = tanh_bounds(p, s, N, M)
    out = np.zeros(len(s))
    for q, row in enumerate(np.asarray(s)):
        _, off = oh.connected(om, row)
        for sp, hv in off:
            d = W @ (sp.astype(np.float64) - row)                 # angle change [M]
            C, S = np.cosh(d), np.sinh(d)
            term = C + t[q] * S
            r = np.exp(a @ (sp - row)) * np.prod(term)
            rel = np.sum((np.abs(S) * dt[q] + 4 * U32 * (np.abs(C) + np.abs(t[q] * S)))
                         / np.abs(term)) + 2 * M * U32
            out[q] += abs(hv * r) * rel
    return out


def jvp_bound(p, s, v, N, M):
    """Bound of |(O v)_s(float) - (O v)_s| per sample."""
    th, t, dt = tanh_bounds(p, s, N, M)
    va, vb, vW = unpack(np.asarray(v), N, M)
    s = np.asarray(s, dtype=np.float64)
    Vs = vb[None, :] + s @ vW.T                                   # [n, M]
    Vabs = np.abs(vb)[None, :] + np.abs(vW).sum(axis=1)[None, :]
    return ((dt * np.abs(Vs)).sum(axis=1) + gamma(N + M + 1) * (np.abs(t) * Vabs).sum(axis=1)
            + gamma(N) * np.abs(va).sum())


def vjp_entries_bound(p, s, u, ks, N, M):
    """Bound of |(O^dagger u)_k(float) - (O^dagger u)_k| for the entries ks."""
    th, t, dt = tanh_bounds(p, s, N, M)
    u = np.abs(np.asarray(u))
    n = len(u)
    per_j = (dt * u[:, None]).sum(axis=0) + gamma(n) * (np.abs(t) * u[:, None]).sum(axis=0)
    out = []
    for k in ks:
        if k < N:
            out.append(gamma(n) * u.sum())
        elif k < N + M:
            out.append(per_j[k - N])
        else:
            out.append(per_j[(k - N - M) // N])
    return np.array(out)
