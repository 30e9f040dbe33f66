"""Oracle: Monte Carlo statistics, energy gradient and stochastic reconfiguration
(test infrastructure only).

Sec. 2.2.5: the energy (Eq. 5) and its gradient are estimated together from the same
samples using the analytic RBM log-derivatives; stochastic reconfiguration (the paper's
"Sr" method, natural-gradient / imaginary-time step) solves a linear system with either
an exact or an iterative solver; the parameters then move as in Eq. 2 with learning rate
lambda. Definitions of the cited SR method, restated with population averages <.> over
the n samples:

    E     = <E_loc>,    var = <|E_loc - E|^2>
    F_k   = <conj(O_k) E_loc> - <conj(O_k)> <E_loc>
    S_kk' = <conj(O_k) O_k'> - <conj(O_k)> <O_k'>
    (S + diag_shift * I) x = F,   p <- p - lr * x.

``cg`` is textbook conjugate gradients for a Hermitian positive-definite operator, x0 = 0,
stopping when ||r|| <= tol * ||F|| or after maxiter matrix-vector products.

Pins (tests/test_oracle_sr.py): ``stats`` against a hand-built layout whose chain means
and variance are known in closed form, and the unbiasedness of err^2 (its average over
many independent Gaussian data sets equals sigma^2 / n); F against finite differences of
the exact energy
(dE/dRe p_k = 2 Re F_k, dE/dIm p_k = 2 Im F_k), the quadratic form v^dagger S v against
the norm of the finite-difference tangent vector projected orthogonally to psi, CG
against a dense solve, and exact-expectation SR descending to the exact ground energy.
"""
import numpy as np

from . import exact, hamiltonian, lattice, rbm


def stats(eloc, n_chains=None):
    """Mean, variance and error bar of the local energies (Sec. 2.2.5: the energy is
    reported with its statistical uncertainty and its variance).

    mean = <E_loc>, var = <|E_loc - mean|^2> (population averages over the n samples).
    The error bar is the standard error of the mean estimated from chain means: the
    samples are laid out [n_sweeps, n_chains] (row-major: sample s = sweep * n_chains +
    chain), m_c is the mean of Re E_loc over chain c's sweeps, and

        err = sqrt( sum_c (m_c - mean(m))^2 / (C - 1) ) / sqrt(C)

    (the unbiased variance of the C chain means, over C). Without a chain count every
    sample is its own chain (C = n, one sweep)."""
    e = np.asarray(eloc)
    n = e.size
    mean = e.mean()
    var = np.mean(np.abs(e - mean) ** 2)
    C = int(n_chains) if n_chains else n
    if C < 2 or n % C:
        raise ValueError("need at least two chains dividing the sample count")
    chain_means = e.real.reshape(n // C, C).mean(axis=0)
    d = chain_means - chain_means.mean()
    err = np.sqrt(np.sum(d * d) / (C - 1)) / np.sqrt(C)
    return mean, var, err


def force(O, eloc, weights=None):
    """F_k = <conj(O_k)(E_loc - E)>; weights = sample probabilities (default 1/n)."""
    O = np.asarray(O)
    e = np.asarray(eloc)
    w = np.full(e.shape[0], 1.0 / e.shape[0]) if weights is None else np.asarray(weights)
    Ob = w @ O
    Eb = w @ e
    return (O - Ob).conj().T @ (w * (e - Eb))


def s_matrix(O, weights=None):
    O = np.asarray(O)
    w = np.full(O.shape[0], 1.0 / O.shape[0]) if weights is None else np.asarray(weights)
    Oc = O - w @ O
    return Oc.conj().T @ (w[:, None] * Oc)


def cg(matvec, b, tol, maxiter):
    """Returns (x, iterations, ||r|| / ||b||)."""
    b = np.asarray(b)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.real(np.vdot(r, r))
    bnorm = np.sqrt(rr)
    if bnorm == 0.0:
        return x, 0, 0.0
    it = 0
    while it < maxiter:
        Ap = matvec(p)
        alpha = rr / np.real(np.vdot(p, Ap))
        x = x + alpha * p
        r = r - alpha * Ap
        it += 1
        rr_new = np.real(np.vdot(r, r))
        if np.sqrt(rr_new) <= tol * bnorm:
            rr = rr_new
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it, np.sqrt(rr) / bnorm


def sr_step(model, params, samples, eloc, lr, diag_shift, cg_tol, cg_maxiter, weights=None,
            round_tanh=None, machine=None):
    """One SR update from samples [n, N] and their local energies [n].
    Returns (new_params, info dict). round_tanh: see rbm.log_derivatives. machine: any
    ansatz with log_derivatives(params, sigma) (default: the RBM of the model)."""
    if machine is None:
        O = rbm.log_derivatives(params, samples, model.n_sites, model.n_hidden, round_tanh)
    else:
        O = machine.log_derivatives(params, samples)
    return sr_step_from_O(O, params, eloc, lr, diag_shift, cg_tol, cg_maxiter, weights)


def sr_step_from_O(O, params, eloc, lr, diag_shift, cg_tol, cg_maxiter, weights=None):
    """The SR update of any ansatz from its log-derivatives O [n, P] at the samples."""
    e = np.asarray(eloc)
    if not np.iscomplexobj(params):
        O = O.real
    F = force(O, e, weights)
    S = s_matrix(O, weights)
    x, it, res = cg(lambda v: S @ v + diag_shift * v, F, cg_tol, cg_maxiter)
    if not np.iscomplexobj(params):
        x = x.real
    w = np.full(e.shape[0], 1.0 / e.shape[0]) if weights is None else np.asarray(weights)
    E = w @ e
    var = w @ np.abs(e - E) ** 2
    return params - lr * x, {"iters": it, "resid": res, "energy": E, "variance": var,
                             "force": F, "x": x}


def exact_sr_step(model, params, lr, diag_shift, cg_tol=1e-12, cg_maxiter=10000):
    """SR with expectations over the full basis weighted by exact |psi|^2 (deterministic)."""
    confs, p = exact.exact_probabilities(model, params)
    e = hamiltonian.local_energy(model, params, confs)
    return sr_step(model, params, confs, e, lr, diag_shift, cg_tol, cg_maxiter, weights=p)
