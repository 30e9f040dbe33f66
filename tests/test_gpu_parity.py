"""GPU parity: every entry point of libnqs against the FP64 oracle on the same seeded
inputs, element by element. Tolerances: 1e-10 relative for FP64 models, 1e-5 relative
for FP32 models (scaled by the magnitude of the compared vector); integer results
(chains, samples, lattices) bit-exact."""
import numpy as np
import pytest
import torch

import cases
from oracle import hamiltonian as oh, rbm as orbm, sampler as osamp, sr as osr

pytestmark = pytest.mark.gpu

DEV = "cuda"
ALL = [c for c in cases.CASES if c not in cases.BIG and c not in cases.BF16]


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def wrap(d):
    return np.angle(np.exp(1j * d))


@pytest.mark.parametrize("name", ALL)
def test_log_psi(lib, name):
    m, om = cases.build(lib, name)
    p = cases.params(name)
    s = cases.configs(name, 301, seed=5)
    got = m.log_psi(to_dev(p), to_dev(s)).cpu().numpy()
    exp = orbm.log_psi(p.astype(np.complex128 if m.is_complex else np.float64), s, om.n_sites, om.n_hidden)
    t = cases.tol(name)
    assert np.all(np.abs(np.real(got) - np.real(exp)) <= t * np.maximum(1.0, np.abs(np.real(exp))))
    if m.is_complex:
        assert np.all(np.abs(wrap(np.imag(got) - np.imag(exp))) <= t * np.maximum(1.0, np.abs(np.imag(exp))))


@pytest.mark.parametrize("name", ALL)
@pytest.mark.parametrize("init", ["paper_init", "trained_scale"])
def test_local_energy(lib, name, init):
    m, om = cases.build(lib, name)
    p = cases.params(name, sigma=0.01, seed=11) if init == "paper_init" else cases.params(name, seed=11)
    s = cases.configs(name, 203, seed=6)
    got = m.local_energy(to_dev(p), to_dev(s)).cpu().numpy()
    exp = oh.local_energy(om, p.astype(np.complex128 if m.is_complex else np.float64), s)
    scale = max(1.0, np.abs(exp).max())
    err = np.abs(got - exp).max()
    assert err <= cases.tol(name) * scale, (err, scale)


def test_local_energy_empty_and_single(lib):
    m, om = cases.build(lib, "heis40_cplx_f64")
    p = to_dev(cases.params("heis40_cplx_f64"))
    empty = torch.empty((0, 40), dtype=torch.int8, device=DEV)
    assert m.local_energy(p, empty).numel() == 0
    s = cases.configs("heis40_cplx_f64", 1, seed=1)
    got = m.local_energy(p, to_dev(s)).cpu().numpy()
    exp = oh.local_energy(om, p.cpu().numpy(), s)
    assert np.abs(got - exp).max() <= 1e-10 * max(1.0, np.abs(exp).max())


@pytest.mark.parametrize("name", ALL)
def test_jvp_vjp(lib, name):
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=21)
    n = 517
    s = cases.configs(name, n, seed=7)
    rng = np.random.default_rng(3)
    P = m.n_params
    if m.is_complex:
        u = rng.normal(size=n) + 1j * rng.normal(size=n)
        v = rng.normal(size=P) + 1j * rng.normal(size=P)
    else:
        u = rng.normal(size=n)
        v = rng.normal(size=P)
    vjp, jvp = m.log_psi_grad(to_dev(p), to_dev(s), u=to_dev(u), v=to_dev(v))
    pe = p.astype(np.complex128 if m.is_complex else np.float64)
    O = orbm.log_derivatives(pe, s, om.n_sites, om.n_hidden)
    if not m.is_complex:
        O = O.real
    ej = O @ v
    ev = O.conj().T @ u
    t = cases.tol(name)
    assert np.abs(jvp.cpu().numpy() - ej).max() <= t * np.abs(ej).max()
    assert np.abs(vjp.cpu().numpy() - ev).max() <= t * np.abs(ev).max()


@pytest.mark.parametrize("name", ["tfim10_real_f64", "heis40_cplx_f64", "j1j2_4x4_cplx_f64", "tfim37_cplx_f64"])
def test_chain_init_bit_exact(lib, name):
    m, om = cases.build(lib, name)
    C = 133
    ch = torch.empty((C, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=99, chain_offset=5)
    exp = osamp.init_chains(om, C, seed=99, chain_offset=5)
    assert np.array_equal(ch.cpu().numpy(), exp)


@pytest.mark.parametrize("name,margin", [("tfim10_real_f64", 1e-12), ("heis40_cplx_f64", 1e-12),
                                         ("j1j2_4x4_cplx_f64", 1e-12), ("tfim37_cplx_f64", 1e-12),
                                         ("j1j2_6x6_cplx_f64", 1e-12), ("heis12_real_f64_flip", 1e-12),
                                         ("heis40_cplx_f32", 1e-4), ("tfim37_real_f32", 1e-4),
                                         ("heis6x6_cplx_f32", 1e-4), ("heis4x4_cplx_f32_m1024", 1e-4),
                                         ("tfim300_real_f32", 1e-4)])
def test_sampling_matches_oracle(lib, name, margin):
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=31)
    C, n_sweeps, n_discard = 24, 6, 3
    ch = torch.empty((C, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=1234)
    init = ch.cpu().numpy().copy()
    nacc = torch.zeros(C, dtype=torch.int64, device=DEV)
    smp, _ = m.sample(to_dev(p), ch, n_sweeps, n_discard, seed=1234, counter=17, n_accepted=nacc)
    ties = []
    exp, last, nacc_o = osamp.sample(om, p.astype(np.complex128 if m.is_complex else np.float64),
                                     init, n_sweeps, n_discard, seed=1234, counter=17,
                                     record_ties=ties, tie_margin=margin)
    got = smp.cpu().numpy()
    diverged = cases.compare_chains(got, exp, ties, n_discard)
    if diverged == 0:
        assert np.array_equal(ch.cpu().numpy(), last)
        assert np.array_equal(nacc.cpu().numpy(), nacc_o)


def test_sampling_resume_is_bit_exact(lib):
    """Two calls of 3 sweeps (counter advanced) equal one call of 6 sweeps."""
    m, om = cases.build(lib, "heis40_cplx_f64")
    p = to_dev(cases.params("heis40_cplx_f64"))
    ch1 = torch.empty((40, 40), dtype=torch.int8, device=DEV)
    m.chain_init(ch1, seed=5)
    ch2 = ch1.clone()
    a, _ = m.sample(p, ch1, 6, 0, seed=5, counter=100)
    b1, _ = m.sample(p, ch2, 3, 0, seed=5, counter=100)
    b2, _ = m.sample(p, ch2, 3, 0, seed=5, counter=103)
    assert torch.equal(a, torch.cat([b1, b2]))
    assert torch.equal(ch1, ch2)


@pytest.mark.parametrize("name", ["tfim10_real_f64", "heis40_cplx_f32", "heis40_cplx_f64", "j1j2_4x4_cplx_f64",
                                  "tfim5x5_j2_real_f64", "heis12_real_f64_flip", "heis6x6_cplx_f32",
                                  "j1j2_6x6_cplx_f64", "heis4x4_cplx_f32_m1024"])
def test_fused_local_energy_matches_oracle(lib, name):
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=41)
    C = 37
    ch = torch.empty((C, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=3)
    smp, el = m.sample(to_dev(p), ch, 3, 2, seed=3, counter=0, with_eloc=True)
    flat = smp.reshape(-1, om.n_sites).cpu().numpy()
    exp = oh.local_energy(om, p.astype(np.complex128 if m.is_complex else np.float64), flat)
    scale = max(1.0, np.abs(exp).max())
    assert np.abs(el.cpu().numpy() - exp).max() <= cases.tol(name) * scale


@pytest.mark.parametrize("name", ["tfim10_real_f64", "heis40_cplx_f32", "j1j2_4x4_cplx_f64", "heis6x6_cplx_f32"])
def test_local_energy_fused_in_sweep(lib, name):
    """With >= 16 chains per compute unit the local energies are evaluated inside the
    sweep kernel; check a random subset of them against the oracle."""
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=42)
    C = 16 * torch.cuda.get_device_properties(0).multi_processor_count
    ch = torch.empty((C, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=4)
    smp, el = m.sample(to_dev(p), ch, 2, 1, seed=4, counter=0, with_eloc=True)
    flat = smp.reshape(-1, om.n_sites).cpu().numpy()
    rows = np.random.default_rng(0).choice(flat.shape[0], 150, replace=False)
    exp = oh.local_energy(om, p.astype(np.complex128 if m.is_complex else np.float64), flat[rows])
    scale = max(1.0, np.abs(exp).max())
    assert np.abs(el.cpu().numpy()[rows] - exp).max() <= cases.tol(name) * scale


@pytest.mark.parametrize("name", ["tfim10_real_f64", "heis40_cplx_f64", "j1j2_4x4_cplx_f64", "tfim5x5_j2_real_f64"])
def test_sr_step_fixed_iterations(lib, name):
    """Both sides run exactly 12 CG products (tol = 0) in FP64. Energy, variance and force
    agree to 1e-10/1e-9; the step agrees to 1e-9 or to 10x the oracle's own CG
    sensitivity to 1e-15 relative product noise, whichever is larger (with n = 700 < P
    for the 40-site case, S + 0.01 I has condition number ~1e4 and 12 CG steps amplify
    rounding to ~1e-6)."""
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=0.5, seed=51)
    n = 700
    s = cases.configs(name, n, seed=8)
    pe = p.astype(np.complex128 if m.is_complex else np.float64)
    el = oh.local_energy(om, pe, s)
    pt = to_dev(p.copy())
    info = m.sr_step(pt, to_dev(s), to_dev(el), lr=0.05, diag_shift=0.01, cg_tol=0.0, cg_maxiter=12)
    p_new, info_o = osr.sr_step(om, pe, s, el, lr=0.05, diag_shift=0.01, cg_tol=0.0, cg_maxiter=12)
    assert info["cg_iters"] == info_o["iters"] == 12
    E = info_o["energy"]
    assert abs(info["energy_re"] - np.real(E)) <= 1e-10 * max(1, abs(E))
    assert abs(info["variance"] - info_o["variance"]) <= 1e-9 * max(1, info_o["variance"])
    assert abs(info["force_norm"] - np.linalg.norm(info_o["force"])) <= 1e-9 * np.linalg.norm(info_o["force"])
    O = orbm.log_derivatives(pe, s, om.n_sites, om.n_hidden)
    if not m.is_complex:
        O = O.real
    tol = max(1e-9, 10 * cases.cg_sensitivity(O, el, 0.01, 12))
    dx = pt.cpu().numpy() - p_new
    assert np.abs(dx).max() <= tol * np.abs(p_new - pe).max()


@pytest.mark.parametrize("name", ["heis40_cplx_f32", "j1j2_4x4_cplx_f32", "tfim37_real_f32",
                                  "tfim37_cplx_f32_m37"])
def test_sr_step_fp32_products(lib, name):
    """FP32 matrix-vector products inside the FP64 CG: the step agrees with the FP64
    oracle to 1e-4 of its size (FP32 rounding, amplified by at most the condition number
    of S + 0.01 I over 12 iterations)."""
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=0.3, seed=52)
    n = 640
    s = cases.configs(name, n, seed=9)
    pe = p.astype(np.complex128 if m.is_complex else np.float64)
    el = oh.local_energy(om, pe, s)
    pt = to_dev(p.copy())
    info = m.sr_step(pt, to_dev(s), to_dev(el), lr=0.05, diag_shift=0.01, cg_tol=0.0, cg_maxiter=12)
    p_new, info_o = osr.sr_step(om, pe, s, el, lr=0.05, diag_shift=0.01, cg_tol=0.0, cg_maxiter=12)
    step_o = p_new - pe
    step_g = pt.cpu().numpy().astype(pe.dtype) - pe
    assert np.abs(step_g - step_o).max() <= 1e-4 * np.abs(step_o).max() + 1e-7


def test_sr_step_converged_and_notconv(lib):
    m, om = cases.build(lib, "tfim10_real_f64")
    p = cases.params("tfim10_real_f64", theta=0.5, seed=53)
    s = cases.configs("tfim10_real_f64", 400, seed=10)
    el = oh.local_energy(om, p, s)
    pt = to_dev(p.copy())
    info = m.sr_step(pt, to_dev(s), to_dev(el), lr=0.05, diag_shift=0.01, cg_tol=1e-10, cg_maxiter=500)
    p_new, info_o = osr.sr_step(om, p, s, el, lr=0.05, diag_shift=0.01, cg_tol=1e-10, cg_maxiter=500)
    # iteration counts at tol 1e-10 move by a few steps with the summation order of S v
    assert info["converged"] == 1 and abs(info["cg_iters"] - info_o["iters"]) <= 3
    assert np.abs(pt.cpu().numpy() - p_new).max() <= 1e-7 * np.abs(p_new - p).max()
    pt2 = to_dev(p.copy())
    info2 = m.sr_step(pt2, to_dev(s), to_dev(el), lr=0.05, diag_shift=0.01, cg_tol=1e-14, cg_maxiter=2)
    assert info2["status"] == 1 and info2["converged"] == 0 and info2["cg_iters"] == 2


def _sv_expected(om, pe, s, v, shift):
    """(S + shift I) v from the oracle's explicit S, and the size of the uncentred
    product O^dagger O v / n that rounding is measured against."""
    O = orbm.log_derivatives(pe, s, om.n_sites, om.n_hidden)
    if not np.iscomplexobj(pe):
        O = O.real
    exp = osr.s_matrix(O) @ v + shift * v
    scale = np.abs(O.conj().T @ (O @ v)).max() / s.shape[0]
    return exp, scale


@pytest.mark.parametrize("name,n", [("tfim10_real_f64", 700), ("heis40_cplx_f64", 700),
                                    ("heis40_cplx_f32", 1000), ("j1j2_4x4_cplx_f32", 333),
                                    ("tfim37_real_f32", 517), ("j1j2_6x6_cplx_f64", 129),
                                    ("tfim37_cplx_f32_m37", 2049), ("heis6x6_cplx_f32", 100)])
def test_sr_matvec(lib, name, n):
    """nqs_sr_matvec against (S + lambda I) v with the oracle's explicit S, for two
    directions in a row on one preparation (the workspace is reused). Complex FP32 cases
    run at their smaller typical |theta| (FP32 rounding of theta is amplified near the
    poles of tanh)."""
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=min(0.5, cases.theta_scale(name)), seed=61)
    pe = p.astype(np.complex128 if m.is_complex else np.float64)
    s = cases.configs(name, n, seed=10)
    st = to_dev(s)
    ws = m.sr_prepare(to_dev(p), st)
    rng = np.random.default_rng(62)
    for shift in (0.01, 0.0):
        v = rng.normal(size=m.n_params)
        if m.is_complex:
            v = v + 1j * rng.normal(size=m.n_params)
        got = m.sr_matvec(st, ws, to_dev(v), diag_shift=shift).cpu().numpy()
        exp, scale = _sv_expected(om, pe, s, v, shift)
        assert np.abs(got - exp).max() <= cases.tol(name) * max(scale, shift * np.abs(v).max())


@pytest.mark.parametrize("name,n", [("heis40_cplx_f32", 3000), ("tfim37_cplx_f32_m37", 777)])
def test_sv_shapes_and_autotune(lib, name, n):
    """Every S v kernel shape the autotuner may pick agrees with the oracle's explicit S;
    the autotuner times them all and keeps one."""
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=cases.theta_scale(name), seed=65)
    pe = p.astype(np.complex128)
    s = cases.configs(name, n, seed=12)
    st = to_dev(s)
    rng = np.random.default_rng(66)
    v = rng.normal(size=m.n_params) + 1j * rng.normal(size=m.n_params)
    exp, scale = _sv_expected(om, pe, s, v, 0.01)
    for pairs in (2, 4):
        m.set_sv_shape(pairs)
        ws = m.sr_prepare(to_dev(p), st)
        got = m.sr_matvec(st, ws, to_dev(v), diag_shift=0.01).cpu().numpy()
        assert np.abs(got - exp).max() <= cases.tol(name) * scale, pairs
    rep = m.autotune(to_dev(p), st)
    assert rep["pairs"] == [2, 4] and all(t > 0 for t in rep["us"])
    ws = m.sr_prepare(to_dev(p), st)
    got = m.sr_matvec(st, ws, to_dev(v), diag_shift=0.01).cpu().numpy()
    assert np.abs(got - exp).max() <= cases.tol(name) * scale


def test_sr_matvec_full_size_sampled(lib):
    """The 40-site Heisenberg ring, complex FP32, alpha = 2, at the full 1024 chains x 200
    sweeps = 204800 samples of the benchmark (same kernels and launch shape): entries of
    S v computed one by one by the oracle (y = O v by chunks, then single columns of
    O^dagger (y - mean y) / n)."""
    name = "heis40_cplx_f32"
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=0.3, seed=63)
    pe = p.astype(np.complex128)
    n = 1024 * 200
    s = cases.configs(name, n, seed=11)
    st = to_dev(s)
    ws = m.sr_prepare(to_dev(p), st)
    rng = np.random.default_rng(64)
    v = rng.normal(size=m.n_params) + 1j * rng.normal(size=m.n_params)
    got = m.sr_matvec(st, ws, to_dev(v), diag_shift=0.01).cpu().numpy()
    y = np.concatenate([orbm.jvp(pe, s[i:i + 8192], v, om.n_sites, om.n_hidden)
                        for i in range(0, n, 8192)])
    N, M = om.n_sites, om.n_hidden
    ks = np.unique(np.concatenate([[0, N - 1, N, N + M - 1, m.n_params - 1],
                                   rng.integers(0, m.n_params, 27)]))
    exp = orbm.vjp_entries(pe, s, y - y.mean(), ks, N, M) / n + 0.01 * v[ks]
    scale = np.abs(orbm.vjp_entries(pe, s, y, ks, N, M)).max() / n
    assert np.abs(got[ks] - exp).max() <= cases.tol(name) * scale


@pytest.mark.parametrize("name,n", [("heis40_cplx_f32", 1024 * 200),
                                    ("heis40_cplx_f32", 1024 * 200 - 37),
                                    ("tfim10_real_f64", 136072)])
def test_local_energy_full_size_sampled(lib, name, n):
    """Local energies at sample counts beyond one sample per lane of the whole chip: the
    40-site Heisenberg ring, complex FP32, alpha = 2, at the benchmark's 204800 samples and
    at a ragged count, and a 10-site real FP64 TFIM ring (two blocks per compute unit) at
    136072; the samples of the last partial grid-stride step are shared by several lanes each (8
    and 16 on 256 compute units); entries of both parts against the oracle."""
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=0.3, seed=65)
    pe = p.astype(np.complex128 if m.is_complex else np.float64)
    s = cases.configs(name, n, seed=66)
    el = m.local_energy(to_dev(p), to_dev(s)).cpu().numpy()
    rng = np.random.default_rng(67)
    ks = np.unique(np.concatenate([np.arange(16), np.arange(n - 96, n),
                                   rng.integers(0, n, 48)]))
    eel = oh.local_energy(om, pe, s[ks])
    assert np.abs(el[ks] - eel).max() <= cases.tol(name) * max(1.0, np.abs(eel).max())


@pytest.mark.parametrize("name", ["heis40_cplx_f32", "tfim10_real_f64", "j1j2_4x4_cplx_f64"])
def test_sr_step_graph_replays_match_direct_launches(lib, name):
    """Chunks of CG iterations replayed from a captured graph (several replays per call,
    with the host reading the solver state between them; the second graph call reuses
    the cached graph) give bitwise the parameters of direct launches."""
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=0.3, seed=91)
    n = 700
    s = cases.configs(name, n, seed=92)
    pe = p.astype(np.complex128 if m.is_complex else np.float64)
    el = to_dev(oh.local_energy(om, pe, s))
    st = to_dev(s)
    ws = torch.empty(m.sr_workspace_bytes(n), dtype=torch.uint8, device=DEV)
    out = []
    for graphs in (False, True, True, False):
        m.set_cg_graphs(graphs)
        pt = to_dev(p.copy())
        info = m.sr_step(pt, st, el, lr=0.05, diag_shift=0.01, cg_tol=1e-14, cg_maxiter=40,
                         workspace=ws)
        torch.cuda.synchronize()
        out.append((pt.cpu().numpy(), info["cg_iters"], info["energy_re"]))
    for q in range(1, 4):
        assert np.array_equal(out[0][0], out[q][0]), q
        assert out[0][1] == out[q][1] == 40
