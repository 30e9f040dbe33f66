"""Rounding bounds of the FP32 network near the poles of its activations (test helper,
float64 numpy).

ln cosh and tanh have poles at Im y = pi/2 (mod pi) on Re y = 0: there f'(y) grows without
bound and the float rounding of y is amplified by |f'(y)|. Away from the poles the FP32
tolerance of the parity tests (1e-5 relative) holds; for the units where |f'(y)| > 2 the
first-order bound below is added. The accumulation of y_j = b_j + sum_k W_jk z_k in float
errs by at most gamma_(n+1) (|b_j| + sum_k |W_jk| |z_k|) (recursive summation, any order,
gamma_n = n u / (1 - n u), u = 2^-24), the activation by 4 u (1 + |f(y)|); errors of the
inputs propagate through |W| and |f'|.
"""
import numpy as np

from oracle import ffnn

U32 = 2.0 ** -24
NEAR = 2.0


def gamma(n):
    return n * U32 / (1.0 - n * U32)


def logpsi_pole_bound(net, p, s):
    """Per configuration: first-order bound of the float log psi error that comes from
    units near a pole (their own rounding, propagated through the later layers)."""
    p = np.asarray(p, dtype=np.complex128)
    ys, zs = net.forward(p, s)
    dz = np.zeros(zs[0].shape)
    for l, ((b, W), a) in enumerate(zip(net.unpack(p), net.acts)):
        aW = np.abs(W)
        mag = np.abs(b)[None, :] + np.abs(zs[l]) @ aW.T
        fp = np.abs(ffnn.act_deriv(a, ys[l]))
        near = fp > NEAR
        own = near * (gamma(net.widths[l] + 1) * mag * fp + 4 * U32 * (1 + np.abs(zs[l + 1])))
        dz = fp * (dz @ aW.T) + own
    return dz.sum(axis=1)


def local_energy_pole_bound(om, net, p, s):
    """Per configuration: sum over connected sigma' of |H e^Delta| (bound(sigma') +
    bound(sigma)), with the log psi bounds above."""
    from oracle import hamiltonian as oh
    p = np.asarray(p, dtype=np.complex128)
    out = np.zeros(len(s))
    b0 = logpsi_pole_bound(net, p, s)
    lp = net.log_psi(p, s)
    for q, row in enumerate(np.asarray(s)):
        _, off = oh.connected(om, row)
        if not off:
            continue
        sps = np.array([sp for sp, _ in off])
        hv = np.array([h for _, h in off])
        lq = net.log_psi(p, sps)
        out[q] = np.sum(np.abs(hv * np.exp(lq - lp[q])) * (logpsi_pole_bound(net, p, sps) + b0[q]))
    return out


def well_conditioned(net, p, s, limit=NEAR):
    """Rows of s whose every unit has |f'(y)| <= limit."""
    ys, _ = net.forward(np.asarray(p, dtype=np.complex128), s)
    ok = np.ones(len(s), dtype=bool)
    for y, a in zip(ys, net.acts):
        ok &= np.all(np.abs(ffnn.act_deriv(a, y)) <= limit, axis=1)
    return ok
