"""GPU parity of the feed-forward network (FFNN, Sec. 2.2.2: dense layers with ln cosh /
tanh activations, log psi = sum of the last layer) against oracle/ffnn.py: log psi, local
energies, the Jacobian products O v and O^dagger u, Metropolis sampling on the same random
stream, the SR step and the supervised step. Tolerances as for the RBM: 1e-10 relative
for FP64, 1e-5 for FP32 (scaled by the magnitude of the compared vector), plus for FP32
the first-order rounding bound of units near a pole of their activation (ff_bounds.py);
FP32 Jacobian products are checked on configurations away from the poles."""
import numpy as np
import pytest
import torch

import cases
import ff_bounds
import synth
from oracle import ffnn, hamiltonian as oh, lattice as ol, sampler as osamp, sr as osr
from oracle import supervised as osup

pytestmark = pytest.mark.gpu

DEV = "cuda"
LC, TH = ffnn.LNCOSH, ffnn.TANH

# name: (L, ndim, diagonals, ham, J, h, marshall, move, complex, prec, layers, activations)
FF = {
    "ff_tfim10_real_f64": (10, 1, False, 0, (1.0, 0.0), 1.0, False, 0, False, 0, [20, 10], [LC, TH]),
    "ff_heis40_cplx_f64": (40, 1, False, 1, (1.0, 0.0), 0.0, True, 1, True, 0, [80, 40], [LC, LC]),
    "ff_heis40_cplx_f32": (40, 1, False, 1, (1.0, 0.0), 0.0, True, 1, True, 1, [80, 40], [LC, LC]),
    "ff_j1j2_4x4_cplx_f64": (4, 2, True, 1, (1.0, 0.5), 0.0, True, 1, True, 0, [32, 16, 8],
                             [TH, LC, LC]),
    "ff_tfim37_cplx_f32": (37, 1, False, 0, (1.0, 0.0), 0.9, False, 0, True, 1, [74, 37], [LC, TH]),
    "ff_tfim12_real_f32_one": (12, 1, False, 0, (1.0, 0.0), 1.1, False, 0, False, 1, [24], [LC]),
    # widest layers (512 outputs, eight per lane) and more sites than any layer is wide
    "ff_heis16_cplx_f32_w512": (16, 1, False, 1, (1.0, 0.0), 0.0, True, 1, True, 1, [512, 64],
                                [LC, TH]),
    "ff_tfim300_cplx_f32": (300, 1, False, 0, (1.0, 0.0), 1.0, False, 0, True, 1, [64, 32],
                            [LC, LC]),
    "ff_heis12_cplx_f64_four": (12, 1, False, 1, (1.0, 0.0), 0.0, True, 1, True, 0,
                                [24, 20, 16, 12], [TH, TH, LC, TH]),
}
SMALL = [k for k in FF if k != "ff_tfim300_cplx_f32"]


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def wrap(d):
    return np.angle(np.exp(1j * d))


def build(lib, name):
    L, ndim, diag, ham, J, h, marshall, move, cplx, prec, layers, acts = FF[name]
    bonds, sub = lib.nqs_hypercube(L, ndim, diag)
    N = L ** ndim
    m = lib.Model(N, layers[0], bonds, ham=ham, J=J, h=h, marshall=marshall, sublattice=sub,
                  move=move, is_complex=cplx, prec=prec, layers=layers, activations=acts)
    ob, osub = ol.hypercube(L, ndim, with_diagonals=diag)
    om = oh.Model(N, layers[0], ob, ham=ham, J=J, h=h, marshall=marshall, sublattice=osub,
                  move=move, is_complex=cplx)
    net = ffnn.FFNN(N, layers, acts)
    assert m.n_params == net.n_params
    return m, om, net


def params(name, net, seed, theta=0.8):
    """Weights of every layer scaled by its fan-in (typical |y| ~ theta), exactly
    representable in the case's precision."""
    prec, cplx = FF[name][9], FF[name][8]
    rng = np.random.default_rng(seed)
    layers = []
    for l in range(len(net.sizes)):
        wi, wo = net.widths[l], net.widths[l + 1]
        s = theta / np.sqrt(wi + 1.0)
        b = rng.normal(0, s, wo) + (1j * rng.normal(0, s, wo) if cplx else 0)
        W = rng.normal(0, s, (wo, wi)) + (1j * rng.normal(0, s, (wo, wi)) if cplx else 0)
        layers.append((b, W))
    p = net.pack(layers)
    if prec == 1:
        p = p.astype(np.complex64 if cplx else np.float32)
    return p


def oracle_p(p):
    return p.astype(np.complex128 if np.iscomplexobj(p) else np.float64)


def configs(name, n, seed):
    L, ndim = FF[name][0], FF[name][1]
    return synth.spin_configs(n, L ** ndim, seed, zero_magnetisation=(FF[name][7] == 1))


def tol(name):
    return 1e-10 if FF[name][9] == 0 else 1e-5


@pytest.mark.parametrize("name", list(FF))
def test_ff_log_psi(lib, name):
    m, om, net = build(lib, name)
    p = params(name, net, seed=1)
    s = configs(name, 333, seed=2)
    lp = m.log_psi(to_dev(p), to_dev(s)).cpu().numpy()
    exp = net.log_psi(oracle_p(p), s)
    scale = max(1.0, np.abs(exp).max())
    bound = 0.0 if m.prec == 0 else 2 * ff_bounds.logpsi_pole_bound(net, p, s)
    assert np.all(np.abs(lp.real - exp.real) <= tol(name) * scale + bound)
    if m.is_complex:
        assert np.all(np.abs(wrap(lp.imag - exp.imag)) <= tol(name) * scale + bound)


@pytest.mark.parametrize("name", list(FF))
def test_ff_local_energy(lib, name):
    m, om, net = build(lib, name)
    p = params(name, net, seed=3)
    n = 40 if name == "ff_tfim300_cplx_f32" else 150
    s = configs(name, n, seed=4)
    el = m.local_energy(to_dev(p), to_dev(s)).cpu().numpy()
    exp = oh.local_energy(om, oracle_p(p), s, machine=net)
    bound = 0.0 if m.prec == 0 else 2 * ff_bounds.local_energy_pole_bound(om, net, p, s)
    assert np.all(np.abs(el - exp) <= tol(name) * max(1.0, np.abs(exp).max()) + bound)


@pytest.mark.parametrize("name", list(FF))
def test_ff_jvp_vjp(lib, name):
    """On configurations whose every unit has |f'(y)| <= 4: near a pole the derivatives
    themselves are ill-conditioned (in FP64 as well), which the log psi and local energy
    tests cover with their bounds."""
    m, om, net = build(lib, name)
    p = params(name, net, seed=5, theta=0.3)
    n = 97 if name == "ff_tfim300_cplx_f32" else 1000   # several sample splits, ragged
    s = configs(name, 3 * n, seed=6)
    s = s[ff_bounds.well_conditioned(net, p, s, limit=4.0)][:n]
    assert len(s) >= n // 2
    n = len(s)
    rng = np.random.default_rng(7)
    P = net.n_params
    v = rng.normal(size=P) + (1j * rng.normal(size=P) if m.is_complex else 0)
    u = rng.normal(size=n) + (1j * rng.normal(size=n) if m.is_complex else 0)
    vjp, jvp = m.log_psi_grad(to_dev(p), to_dev(s), u=to_dev(u), v=to_dev(v))
    O = net.log_derivatives(oracle_p(p), s)
    if not m.is_complex:
        O = O.real
    ej, ev = O @ v, np.conj(O).T @ u
    assert np.abs(jvp.cpu().numpy() - ej).max() <= tol(name) * np.abs(ej).max()
    assert np.abs(vjp.cpu().numpy() - ev).max() <= tol(name) * np.abs(ev).max()


@pytest.mark.parametrize("name,margin", [("ff_tfim10_real_f64", 1e-12), ("ff_heis40_cplx_f64", 1e-12),
                                         ("ff_j1j2_4x4_cplx_f64", 1e-12),
                                         ("ff_heis12_cplx_f64_four", 1e-12),
                                         ("ff_heis40_cplx_f32", 1e-3), ("ff_tfim37_cplx_f32", 1e-3),
                                         ("ff_tfim12_real_f32_one", 1e-3),
                                         ("ff_heis16_cplx_f32_w512", 1e-3)])
def test_ff_sampling_matches_oracle(lib, name, margin):
    """FP32 decisions take a margin of 1e-3: the float log psi errs by up to ~1e-4 near the
    activations' poles (ff_bounds.py)."""
    m, om, net = build(lib, name)
    p = params(name, net, seed=8, theta=0.3)
    C, S, D = 20, 4, 2
    ch = torch.empty((C, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=31)
    init = ch.cpu().numpy().copy()
    nacc = torch.zeros(C, dtype=torch.int64, device=DEV)
    smp, el = m.sample(to_dev(p), ch, S, D, seed=77, counter=5, chain_offset=2, n_accepted=nacc,
                       with_eloc=True)
    ties = []
    exp, last, nacc_o = osamp.sample(om, oracle_p(p), init, S, D, seed=77, counter=5,
                                     chain_offset=2, record_ties=ties, tie_margin=margin,
                                     machine=net)
    got = smp.cpu().numpy()
    if cases.compare_chains(got, exp, ties, D) == 0:
        assert np.array_equal(ch.cpu().numpy(), last)
        assert np.array_equal(nacc.cpu().numpy(), nacc_o)
    flat = got.reshape(-1, om.n_sites)
    ee = oh.local_energy(om, oracle_p(p), flat, machine=net)
    bound = 0.0 if m.prec == 0 else 2 * ff_bounds.local_energy_pole_bound(om, net, p, flat)
    assert np.all(np.isfinite(ee))
    err = np.abs(el.cpu().numpy() - ee)
    lim = tol(name) * np.maximum(1.0, np.abs(ee)) + bound
    q = int(np.argmax(err / lim))
    assert err[q] <= lim[q], (q, err[q], lim[q], ee[q], el.cpu().numpy()[q])


@pytest.mark.parametrize("name", ["ff_tfim10_real_f64", "ff_heis40_cplx_f64", "ff_j1j2_4x4_cplx_f64",
                                  "ff_heis12_cplx_f64_four"])
def test_ff_sr_step(lib, name):
    """The SR step of the network: fixed 12 CG iterations against the oracle's CG on the
    same samples, energies and shift."""
    m, om, net = build(lib, name)
    p = params(name, net, seed=9, theta=0.3)
    s = configs(name, 512, seed=10)
    pe = oracle_p(p)
    el = oh.local_energy(om, pe, s, machine=net)
    pt = to_dev(p.copy())
    info = m.sr_step(pt, to_dev(s), to_dev(el), lr=0.05, diag_shift=0.01, cg_tol=0.0,
                     cg_maxiter=12, n_chains=16)
    p_new, io = osr.sr_step(om, pe, s, el, lr=0.05, diag_shift=0.01, cg_tol=0.0, cg_maxiter=12,
                            machine=net)
    assert info["cg_iters"] == io["iters"] == 12
    assert abs(info["energy_re"] - np.real(io["energy"])) <= 1e-10 * max(1, abs(io["energy"]))
    assert abs(info["force_norm"] - np.linalg.norm(io["force"])) <= 1e-9 * np.linalg.norm(io["force"])
    # finite-precision CG amplifies rounding with the condition number of S + 0.01 I
    O = net.log_derivatives(pe, s)
    if not m.is_complex:
        O = O.real
    t = max(1e-9, 10 * cases.cg_sensitivity(O, el, 0.01, 12))
    step_o = p_new - pe
    step_g = pt.cpu().numpy() - pe
    assert np.abs(step_g - step_o).max() <= t * np.abs(step_o).max()


@pytest.mark.parametrize("name", ["ff_heis40_cplx_f32", "ff_tfim37_cplx_f32"])
def test_ff_sr_step_fp32_and_async(lib, name):
    """FP32 products inside the FP64 CG agree with the FP64 oracle to 1e-4 of the step, or
    to ten times the CG's amplification of 1e-6 relative product errors when that is larger
    (the condition of S + 0.01 I); the stream-ordered entry point gives the synchronising
    one's parameters bit for bit."""
    m, om, net = build(lib, name)
    p = params(name, net, seed=11, theta=0.4)
    s = configs(name, 640, seed=12)
    pe = oracle_p(p)
    el = oh.local_energy(om, pe, s, machine=net)
    pt = to_dev(p.copy())
    m.sr_step(pt, to_dev(s), to_dev(el), lr=0.05, diag_shift=0.01, cg_tol=0.0, cg_maxiter=12)
    p_new, _ = osr.sr_step(om, pe, s, el, lr=0.05, diag_shift=0.01, cg_tol=0.0, cg_maxiter=12,
                           machine=net)
    O = net.log_derivatives(pe, s)
    t = max(1e-4, 10 * cases.cg_sensitivity(O if m.is_complex else O.real, el, 0.01, 12, rel=1e-6))
    step_o = p_new - pe
    step_g = pt.cpu().numpy().astype(pe.dtype) - pe
    assert np.abs(step_g - step_o).max() <= t * np.abs(step_o).max() + 1e-7
    pa = to_dev(p.copy())
    buf = m.sr_step_async(pa, to_dev(s), to_dev(el), lr=0.05, diag_shift=0.01, cg_tol=0.0,
                          cg_maxiter=12)
    torch.cuda.synchronize()
    assert torch.equal(pa, pt)
    pc = to_dev(p.copy())
    info_c = m.sr_step(pc, to_dev(s), to_dev(el), lr=0.05, diag_shift=0.01, cg_tol=1e-6,
                       cg_maxiter=300)
    assert info_c["converged"] == 1


def test_ff_one_layer_is_the_rbm_on_the_gpu(lib):
    """One ln cosh layer and the RBM with zero visible bias give the same amplitudes and
    local energies (two different kernels)."""
    name = "ff_tfim12_real_f32_one"
    m, om, net = build(lib, name)
    p = params(name, net, seed=13)
    (b, W), = net.unpack(p)
    bonds, sub = lib.nqs_hypercube(12, 1)
    r = lib.Model(12, 24, bonds, ham=0, J=(1.0, 0.0), h=1.1, is_complex=False, prec=1)
    pr = np.concatenate([np.zeros(12, dtype=np.float32), b, W.reshape(-1)])
    s = configs(name, 200, seed=14)
    a1 = m.log_psi(to_dev(p), to_dev(s)).cpu().numpy()
    a2 = r.log_psi(to_dev(pr), to_dev(s)).cpu().numpy()
    assert np.abs(a1 - a2).max() <= 1e-5 * np.abs(a2).max()
    e1 = m.local_energy(to_dev(p), to_dev(s)).cpu().numpy()
    e2 = r.local_energy(to_dev(pr), to_dev(s)).cpu().numpy()
    assert np.abs(e1 - e2).max() <= 1e-5 * np.abs(e2).max()


def test_ff_overlap_step(lib):
    name = "ff_heis40_cplx_f64"
    m, om, net = build(lib, name)
    p = params(name, net, seed=15, theta=0.5)
    s = configs(name, 500, seed=16)
    rng = np.random.default_rng(17)
    lt = rng.normal(0, 0.5, 500) + 1j * rng.uniform(-np.pi, np.pi, 500)
    pd = to_dev(p.copy())
    info = m.overlap_step(pd, to_dev(s), to_dev(lt), 0.1)
    loss, g, _ = osup.estimator(net.log_psi(p, s), lt, net.log_derivatives(p, s))
    assert abs(info["loss"] - loss) <= 1e-10 * max(1.0, abs(loss))
    assert np.abs(pd.cpu().numpy() - (p - 0.1 * g)).max() <= 1e-10 * 0.1 * np.abs(g).max()


def test_ff_rejections(lib):
    bonds, sub = lib.nqs_hypercube(8, 1)
    for layers, acts, prec, status in (([8, 8, 8, 8, 8], None, 0, lib.EINVAL),
                                       ([513], None, 0, lib.EINVAL),
                                       ([8], [2], 0, lib.EINVAL),
                                       ([8, 4], None, 2, lib.EUNSUPPORTED)):
        with pytest.raises(lib.NQSError) as ex:
            lib.Model(8, 8, bonds, ham=0, prec=prec, layers=layers, activations=acts)
        assert ex.value.status == status
    m, om, net = build(lib, "ff_heis40_cplx_f32")
    p = to_dev(params("ff_heis40_cplx_f32", net, seed=1))
    reps = torch.ones((2, 2, 40), dtype=torch.int8, device=DEV)
    tix = torch.zeros((2, 2), dtype=torch.int32, device=DEV)
    with pytest.raises(lib.NQSError) as ex:
        m.sample_pt(p, reps, tix, 1, 0, seed=1, counter=0)
    assert ex.value.status == lib.EUNSUPPORTED
