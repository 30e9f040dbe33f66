"""Parity cases: one lattice model + RBM shape + precision, built twice - once as a
library handle, once as an oracle model - from the same description."""
import numpy as np

import synth
from oracle import hamiltonian as oh
from oracle import sr as osr
from oracle import lattice as ol

# name: (L, ndim, diagonals, ham, J, h, marshall, move, complex, prec, M)
# prec: 0 = FP64, 1 = FP32, 2 = BF16
CASES = {
    # 1D TFIM, N = 10, real FP64 RBM, alpha = 1
    "tfim10_real_f64": (10, 1, False, 0, (1.0, 0.0), 1.0, False, 0, False, 0, 10),
    # 1D Heisenberg, N = 40, Marshall sign, exchange moves, complex FP32, alpha = 2
    "heis40_cplx_f32": (40, 1, False, 1, (1.0, 0.0), 0.0, True, 1, True, 1, 80),
    "heis40_cplx_f64": (40, 1, False, 1, (1.0, 0.0), 0.0, True, 1, True, 0, 80),
    # 2D J1-J2, 4x4, J2 = 0.5, complex, alpha = 4
    "j1j2_4x4_cplx_f64": (4, 2, True, 1, (1.0, 0.5), 0.0, True, 1, True, 0, 64),
    "j1j2_4x4_cplx_f32": (4, 2, True, 1, (1.0, 0.5), 0.0, True, 1, True, 1, 64),
    # ragged sizes: N = 37 ring, M = 74; 5x5 TFIM with a J2 term
    "tfim37_real_f32": (37, 1, False, 0, (1.0, 0.0), 0.8, False, 0, False, 1, 74),
    "tfim37_cplx_f64": (37, 1, False, 0, (1.0, 0.0), 1.3, False, 0, True, 0, 74),
    "tfim37_cplx_f32_m37": (37, 1, False, 0, (1.0, 0.0), 0.9, False, 0, True, 1, 37),
    "tfim5x5_j2_real_f64": (5, 2, True, 0, (1.0, -0.3), 1.1, False, 0, False, 0, 50),
    # Heisenberg without Marshall rotation, single flips, real FP64
    "heis12_real_f64_flip": (12, 1, False, 1, (1.0, 0.0), 0.0, False, 0, False, 0, 36),
    # tables too large for LDS (global rows, next-row prefetch), 4 hidden units per lane
    "heis6x6_cplx_f32": (6, 2, False, 1, (1.0, 0.0), 0.0, True, 1, True, 1, 144),
    "j1j2_6x6_cplx_f64": (6, 2, True, 1, (1.0, 0.5), 0.0, True, 1, True, 0, 72),
    # 16 hidden units per lane
    "heis4x4_cplx_f32_m1024": (4, 2, False, 1, (1.0, 0.0), 0.0, True, 1, True, 1, 1024),
}

# larger lattices used by selected tests only (the oracle is slow for them)
BIG = {
    # more than 256 sites: spins read from LDS instead of lane registers
    "tfim300_real_f32": (300, 1, False, 0, (1.0, 0.0), 1.0, False, 0, False, 1, 300),
    # the same with at most 256 hidden units (tempered sweeps)
    "tfim300_cplx_f32_m150": (300, 1, False, 0, (1.0, 0.0), 1.0, False, 0, True, 1, 150),
    # site counts beyond one LDS window of the FP32 Jacobian-vector kernel for each of its
    # block shapes (one, two and four hidden chunks per block)
    "tfim100_cplx_f32_m32": (100, 1, False, 0, (1.0, 0.0), 1.0, False, 0, True, 1, 32),
    "tfim150_cplx_f32_m100": (150, 1, False, 0, (1.0, 0.0), 0.7, False, 0, True, 1, 100),
    # the 10x10 J1-J2 lattice with alpha = 4 and the 16x16 Heisenberg lattice with
    # alpha = 8 of the large workloads
    "j1j2_10x10_cplx_f32": (10, 2, True, 1, (1.0, 0.5), 0.0, True, 1, True, 1, 400),
    "heis16x16_cplx_f32": (16, 2, False, 1, (1.0, 0.0), 0.0, True, 1, True, 1, 2048),
}
BIG_BF16 = {
    "j1j2_10x10_cplx_bf16": (10, 2, True, 1, (1.0, 0.5), 0.0, True, 1, True, 2, 400),
    "heis16x16_cplx_bf16": (16, 2, False, 1, (1.0, 0.0), 0.0, True, 1, True, 2, 2048),
}
BIG.update(BIG_BF16)
CASES.update(BIG)

# BF16 form (prec 2): weights rounded to bfloat16, tanh(theta) rounded for the Jacobian
# contractions, FP32 arithmetic; compared with the oracle running the same quantised
# model (oracle.quant), so the FP32 tolerance applies
BF16 = {
    "heis40_cplx_bf16": (40, 1, False, 1, (1.0, 0.0), 0.0, True, 1, True, 2, 80),
    "j1j2_4x4_cplx_bf16": (4, 2, True, 1, (1.0, 0.5), 0.0, True, 1, True, 2, 64),
    "tfim37_real_bf16": (37, 1, False, 0, (1.0, 0.0), 0.8, False, 0, False, 2, 74),
}
CASES.update(BF16)

TOL = {0: 1e-10, 1: 1e-5, 2: 1e-5}


def build(nqs, name):
    L, ndim, diag, ham, J, h, marshall, move, cplx, prec, M = CASES[name]
    bonds, sub = nqs.nqs_hypercube(L, ndim, diag)
    N = L ** ndim
    lib_model = nqs.Model(N, M, bonds, ham=ham, J=J, h=h, marshall=marshall, sublattice=sub,
                          move=move, is_complex=cplx, prec=prec)
    ob, osub = ol.hypercube(L, ndim, with_diagonals=diag)
    orc = oh.Model(N, M, ob, ham=ham, J=J, h=h, marshall=marshall, sublattice=osub, move=move,
                   is_complex=cplx)
    return lib_model, orc


def theta_scale(name):
    """Typical |theta| the parity tests drive the case at. Complex FP32 cases stay at
    |theta| ~ 0.3: near the zeros of cosh(theta) (Im theta = pi/2) the rounding of theta
    to FP32 alone moves log psi, E_loc and tanh(theta) by more than 1e-5 relative, so the
    FP32 tolerance is stated for theta away from them. FP64 and real cases run at ~1.5."""
    L, ndim, diag, ham, J, h, marshall, move, cplx, prec, M = CASES[name]
    return 0.3 if (cplx and prec >= 1) else 1.5


def params(name, sigma=None, seed=1234, theta=None):
    """Parameters exactly representable in the case's precision. Either sigma (standard
    deviation of every entry) or theta (typical |theta_j|; sigma = theta / sqrt(N + 1))."""
    L, ndim, diag, ham, J, h, marshall, move, cplx, prec, M = CASES[name]
    N = L ** ndim
    if sigma is None:
        sigma = (theta if theta is not None else theta_scale(name)) / np.sqrt(N + 1.0)
    p = synth.rbm_params(N, M, cplx, sigma=sigma, seed=seed)
    if prec >= 1:
        p = p.astype(np.complex64 if cplx else np.float32)
    return p


def oracle_params(name, p):
    """The parameters the oracle evaluates for this case: double precision, with W
    rounded to bfloat16 for the BF16 form."""
    from oracle import quant
    L, ndim, diag, ham, J, h, marshall, move, cplx, prec, M = CASES[name]
    pe = np.asarray(p).astype(np.complex128 if cplx else np.float64)
    return quant.quantize_weights(pe, L ** ndim, M) if prec == 2 else pe


def round_tanh(name):
    """Rounding the case's Jacobian contractions apply to tanh(theta) (BF16 form)."""
    from oracle import quant
    return quant.bf16 if CASES[name][9] == 2 else None


def configs(name, n, seed):
    L, ndim, diag, ham, J, h, marshall, move, cplx, prec, M = CASES[name]
    return synth.spin_configs(n, L ** ndim, seed, zero_magnetisation=(move == 1))


def tol(name):
    return TOL[CASES[name][9]]


def compare_chains(got, exp, ties, n_discard):
    """Recorded samples [S, C, N] equal bit for bit, except that chain c may differ from
    the first sample recorded at or after one of its own near-ties (ties: the oracle's
    (chain, sweep of the call, step) list). Returns the number of chains that differ."""
    diverged = 0
    for c in range(got.shape[1]):
        bad = np.nonzero(np.any(got[:, c] != exp[:, c], axis=1))[0]
        if bad.size:
            assert any(tc == c and sw - n_discard <= bad[0] for tc, sw, _ in ties), (c, bad[0])
            diverged += 1
    return diverged


def cg_sensitivity(O, el, shift, iters, rel=1e-15, seed=0):
    """How far the oracle's own CG result moves when every matrix-vector product is
    perturbed by `rel` relative noise: finite-precision CG amplifies rounding by a factor
    that grows with the condition number of S + shift I."""
    F = osr.force(O, el)
    A = osr.s_matrix(O) + shift * np.eye(O.shape[1])
    x0, _, _ = osr.cg(lambda v: A @ v, F, 0.0, iters)
    rng = np.random.default_rng(seed)
    x1, _, _ = osr.cg(lambda v: (A @ v) * (1 + rel * rng.normal(size=v.shape)), F, 0.0, iters)
    return np.abs(x1 - x0).max() / np.abs(x0).max()
