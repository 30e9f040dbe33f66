"""Oracle: supervised learning by the negative log overlap (test infrastructure only).

Sec. 2.2.3 of the paper: given a target state |t> and the variational state |psi(alpha)>,
the loss of Eq. 1 is

    L(alpha) = -log( <t|psi><psi|t> / (<t|t> <psi|psi>) ),

estimated by Monte Carlo from configurations drawn directly from the target's
distribution |t(sigma)|^2 / <t|t>, and minimised by the update of Eq. 2,
alpha <- alpha - lambda grad L.

Definitions written out here (the paper gives Eq. 1 and Eq. 2 only):

* With R(sigma) = psi(sigma) / t(sigma) and expectations <.>_t over |t|^2,
  <t|psi>/<t|t> = <R>_t and <psi|psi>/<t|t> = <|R|^2>_t, so
  L = -log( |<R>_t|^2 / <|R|^2>_t ).
* psi is holomorphic in alpha with O_k = d log psi / d alpha_k. Then
  d log<psi|psi> / d conj(alpha_k) = <conj(O_k)>_psi = <|R|^2 conj(O_k)>_t / <|R|^2>_t and
  d log<psi|t> / d conj(alpha_k) = <conj(R) conj(O_k)>_t / <conj(R)>_t, while <t|psi> does not
  depend on conj(alpha). The gradient used in Eq. 2 is g = dL / d conj(alpha):
  g_k = sum_s conj(O_sk) u_s,  u_s = |R_s|^2 / sum |R|^2 - conj(R_s) / sum conj(R)
  (reading: for complex parameters the derivative by the conjugate, which is half the
  gradient over real and imaginary parts; for real parameters its real part, half of
  dL/dalpha; the same convention as the force of the SR step).
* Direct sampling of the target over a training set of configurations (all 2^N basis
  states, as in the paper's example): inverse CDF of the cumulative sums of
  |t|^2 (scaled by the largest |t|^2) with one Philox uniform per draw, counter
  (draw, counter, 0, tag 3); the drawn index is the first k with cdf_k > u cdf_last.

Pins (tests/test_oracle_supervised.py): the estimator weighted by the exact |t|^2 over all
states equals the loss and gradient computed from the definition (full sums of t and
psi); the gradient against central finite differences of the exact loss; L = 0 and
g = 0 when psi is proportional to t; the draws against |t|^2 (chi-square); a small SGD
step lowers the exact loss.
"""
import numpy as np

from . import lattice, philox, rbm

TAG_TARGET = 3


def exact_loss(log_psi_all, log_t_all):
    """Eq. 1 from full sums over the training set (both in the same basis order)."""
    lp = np.asarray(log_psi_all, dtype=np.complex128)
    lt = np.asarray(log_t_all, dtype=np.complex128)
    psi = np.exp(lp - lp.real.max())
    t = np.exp(lt - lt.real.max())
    tp = np.vdot(t, psi)                      # <t|psi>
    return float(-np.log((tp * np.conj(tp)).real / (np.vdot(t, t).real * np.vdot(psi, psi).real)))


def exact_gradient(log_psi_all, log_t_all, O_all, real_params=False):
    """g = dL/dconj(alpha) from the full sums: <conj O>_psi - sum conj(psi) t conj(O) /
    sum conj(psi) t."""
    lp = np.asarray(log_psi_all, dtype=np.complex128)
    lt = np.asarray(log_t_all, dtype=np.complex128)
    psi = np.exp(lp - lp.real.max())
    t = np.exp(lt - lt.real.max())
    Oc = np.conj(np.asarray(O_all, dtype=np.complex128))
    p2 = np.abs(psi) ** 2
    g = (p2 @ Oc) / p2.sum() - ((np.conj(psi) * t) @ Oc) / np.sum(np.conj(psi) * t)
    return g.real if real_params else g


def estimator(log_psi_s, log_t_s, O_s, weights=None, real_params=False):
    """Monte Carlo loss and gradient from configurations drawn from |t|^2 (weights: optional
    per-sample weights, 1 by default). Returns (loss, g, u)."""
    d = np.asarray(log_psi_s, dtype=np.complex128) - np.asarray(log_t_s, dtype=np.complex128)
    w = np.ones(len(d)) if weights is None else np.asarray(weights, dtype=np.float64)
    R = np.exp(d - d.real.max())              # psi / t up to one common factor
    S1 = np.sum(w * np.abs(R) ** 2)
    S2 = np.sum(w * np.conj(R))
    loss = float(-np.log(np.abs(S2) ** 2 / (w.sum() * S1)))
    u = w * (np.abs(R) ** 2 / S1 - np.conj(R) / S2)
    g = np.conj(np.asarray(O_s, dtype=np.complex128)).T @ u
    return loss, (g.real if real_params else g), u


def target_cdf(log_t_all):
    """Cumulative sums of |t|^2 / max |t|^2 in basis order (sequential, double)."""
    lt = np.asarray(log_t_all, dtype=np.complex128)
    p = np.exp(2.0 * (lt.real - lt.real.max()))
    return np.cumsum(p)


def draw(cdf, n, seed, counter):
    """Indices of n direct draws from the target distribution."""
    w = philox.draw(seed, np.arange(n, dtype=np.uint64), counter, 0, TAG_TARGET)
    u = philox.uniform_from_words(w[:, 1], w[:, 2])
    x = u * cdf[-1]
    return np.searchsorted(cdf, x, side="right").astype(np.int64)


def near_ties(cdf, n, seed, counter, margin=1e-12):
    """Draws whose scaled uniform lies within margin * cdf_last of a cumulative sum."""
    w = philox.draw(seed, np.arange(n, dtype=np.uint64), counter, 0, TAG_TARGET)
    x = philox.uniform_from_words(w[:, 1], w[:, 2]) * cdf[-1]
    k = np.searchsorted(cdf, x, side="right")
    lo = np.abs(x - cdf[np.clip(k - 1, 0, len(cdf) - 1)])
    hi = np.abs(cdf[np.clip(k, 0, len(cdf) - 1)] - x)
    return np.nonzero(np.minimum(lo, hi) < margin * cdf[-1])[0]


def rbm_step(params, sigma, log_t_s, n_sites, n_hidden, lr):
    """One update of Eq. 2 for the RBM from target-distributed samples.
    Returns (new params, loss estimate, g)."""
    p = np.asarray(params)
    real = not np.iscomplexobj(p)
    lp = rbm.log_psi(p, sigma, n_sites, n_hidden)
    O = rbm.log_derivatives(p, sigma, n_sites, n_hidden)
    loss, g, _ = estimator(lp, log_t_s, O, real_params=real)
    return p - lr * g, loss, g


def rbm_exact(params, log_t_all, n_sites, n_hidden):
    """Exact loss and gradient of the RBM over all 2^N states (lattice.all_configs order)."""
    p = np.asarray(params)
    confs = lattice.all_configs(n_sites)
    lp = rbm.log_psi(p, confs, n_sites, n_hidden)
    O = rbm.log_derivatives(p, confs, n_sites, n_hidden)
    return (exact_loss(lp, log_t_all),
            exact_gradient(lp, log_t_all, O, real_params=not np.iscomplexobj(p)))
