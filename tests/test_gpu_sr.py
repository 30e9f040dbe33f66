"""GPU checks of the SR step beyond single-call parity: the energy error bar against the
oracle's chain-mean estimate, the stream-ordered entry points against the synchronising
ones (bit for bit), replays of captured graphs against direct launches, and the
non-finite contract (status ENONFINITE, parameters unchanged bit for bit)."""
import numpy as np
import pytest
import torch

import cases
import synth
from oracle import hamiltonian as oh, sr as osr

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def sampled(lib, name, C, S, seed, theta=0.5):
    """Chains sampled by the library: samples [S * C, N] laid out [sweeps, chains] and
    their local energies (double / complex double), parameters as numpy."""
    m, om = cases.build(lib, name)
    p = cases.params(name, theta=theta, seed=seed)
    ch = torch.empty((C, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=seed)
    smp, el = m.sample(to_dev(p), ch, S, 5, seed=seed, counter=0, with_eloc=True)
    return m, om, p, smp.view(S * C, om.n_sites), el


@pytest.mark.parametrize("name", ["tfim10_real_f64", "heis40_cplx_f32", "j1j2_4x4_cplx_f64"])
def test_energy_error_bar_matches_oracle(lib, name):
    C, S = 48, 25
    m, om, p, smp, el = sampled(lib, name, C, S, seed=71)
    e = el.cpu().numpy()
    for nch in (C, 0):
        pt = to_dev(p.copy())
        info = m.sr_step(pt, smp, el, lr=0.01, diag_shift=0.01, cg_tol=1e-8, cg_maxiter=50,
                         n_chains=nch)
        mean, var, err = osr.stats(e, n_chains=nch or None)
        assert abs(info["energy_re"] - mean.real) <= 1e-12 * max(1.0, abs(mean))
        assert abs(info["variance"] - var) <= 1e-10 * max(1.0, var)
        assert abs(info["energy_err"] - err) <= 1e-9 * err, (nch, info["energy_err"], err)
    # chain counts that do not divide the samples, or a single chain, are rejected
    for bad in (7, 1, S * C + 2):
        with pytest.raises(lib.NQSError) as ex:
            m.sr_step(to_dev(p.copy()), smp, el, lr=0.01, diag_shift=0.01, cg_tol=1e-8,
                      cg_maxiter=5, n_chains=bad)
        assert ex.value.status == lib.EINVAL


@pytest.mark.parametrize("name,graphs", [("tfim10_real_f64", True), ("heis40_cplx_f32", True),
                                         ("heis40_cplx_f32", False), ("j1j2_4x4_cplx_f64", True),
                                         ("j1j2_10x10_cplx_bf16", True)])
def test_async_step_equals_synchronising_step(lib, name, graphs):
    """nqs_sr_step_async (cg_maxiter slots, convergence on the device) gives bitwise the
    parameters and the information of nqs_sr_step, converged or stopped at the limit."""
    C, S = 64, 12
    m, om, p, smp, el = sampled(lib, name, C, S, seed=72, theta=0.3)
    m.set_cg_graphs(graphs)
    ws = torch.empty(m.sr_workspace_bytes(S * C), dtype=torch.uint8, device=DEV)
    for tol, maxiter in ((1e-6, 300), (1e-14, 21)):
        ps = to_dev(p.copy())
        i_s = m.sr_step(ps, smp, el, lr=0.02, diag_shift=0.01, cg_tol=tol, cg_maxiter=maxiter,
                        workspace=ws, n_chains=C)
        pa = to_dev(p.copy())
        buf = m.sr_step_async(pa, smp, el, lr=0.02, diag_shift=0.01, cg_tol=tol,
                              cg_maxiter=maxiter, workspace=ws, n_chains=C)
        torch.cuda.synchronize()
        i_a = lib.sr_infos_from_device(buf)[0]
        assert torch.equal(ps, pa), (tol, maxiter)
        # the residual ratio is formed on the host in one path and on the device in the
        # other (square roots may differ in the last bit); everything else is identical
        ra, rs = i_a.pop("cg_resid"), i_s.pop("cg_resid")
        assert abs(ra - rs) <= 1e-15 * max(abs(rs), 1e-300)
        assert i_a == i_s, (i_a, i_s)
        if maxiter == 21:
            assert i_a["status"] == lib.ENOTCONV and i_a["cg_iters"] == 21
        else:
            assert i_a["status"] == lib.OK and i_a["converged"] == 1


@pytest.mark.parametrize("name", ["heis40_cplx_f32", "tfim10_real_f64"])
def test_async_step_graph_replays(lib, name):
    """The stream-ordered step captured into a torch CUDA graph: each replay advances the
    parameters exactly as a direct call does (three replays, compared after each one, with
    the program's own work and synchronisation between them)."""
    C, S = 64, 10
    m, om, p, smp, el = sampled(lib, name, C, S, seed=73, theta=0.3)
    ws = torch.empty(m.sr_workspace_bytes(S * C), dtype=torch.uint8, device=DEV)
    info = torch.zeros(lib.SR_INFO_BYTES, dtype=torch.uint8, device=DEV)
    pg = to_dev(p.copy())
    # one uncaptured call first (one-time kernel attribute set-up), on a scratch copy
    m.sr_step_async(to_dev(p.copy()), smp, el, lr=0.02, diag_shift=0.01, cg_tol=1e-7,
                    cg_maxiter=64, workspace=ws, n_chains=C, info=info)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g, stream=s2):
            m.sr_step_async(pg, smp, el, lr=0.02, diag_shift=0.01, cg_tol=1e-7, cg_maxiter=64,
                            workspace=ws, n_chains=C, info=info)
    torch.cuda.synchronize()
    pd = to_dev(p.copy())
    pg.copy_(pd)
    wsd = torch.empty_like(ws)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        ig = lib.sr_infos_from_device(info)[0]
        b2 = m.sr_step_async(pd, smp, el, lr=0.02, diag_shift=0.01, cg_tol=1e-7, cg_maxiter=64,
                             workspace=wsd, n_chains=C)
        torch.cuda.synchronize()
        idd = lib.sr_infos_from_device(b2)[0]
        assert torch.equal(pg, pd), rep
        assert ig == idd, (rep, ig, idd)
        # unrelated eager work between replays
        _ = (pd.abs() * 2).sum().item()


@pytest.mark.parametrize("name", ["tfim10_real_f64", "heis40_cplx_f32"])
@pytest.mark.parametrize("where", ["eloc", "params"])
def test_nonfinite_step_leaves_params_unchanged(lib, name, where):
    """A NaN in the local energies or in the parameters: status ENONFINITE from both
    entry points, the parameters unchanged bit for bit (the kernels compute normally; the
    non-finite values are supplied from the host)."""
    C, S = 32, 8
    m, om, p, smp, el = sampled(lib, name, C, S, seed=74, theta=0.3)
    if where == "eloc":
        el = el.clone()
        el[5] = float("nan")
    else:
        p = p.copy()
        p[om.n_sites + 3] = np.nan
    p0 = to_dev(p.copy())
    ps = to_dev(p.copy())
    info = m.sr_step(ps, smp, el, lr=0.02, diag_shift=0.01, cg_tol=1e-8, cg_maxiter=30,
                     n_chains=C)
    assert info["status"] == lib.ENONFINITE
    assert torch.equal(ps.view(torch.uint8), p0.view(torch.uint8))
    pa = to_dev(p.copy())
    buf = m.sr_step_async(pa, smp, el, lr=0.02, diag_shift=0.01, cg_tol=1e-8, cg_maxiter=30,
                          n_chains=C)
    torch.cuda.synchronize()
    assert lib.sr_infos_from_device(buf)[0]["status"] == lib.ENONFINITE
    assert torch.equal(pa.view(torch.uint8), p0.view(torch.uint8))


def _tfim_batch(lib, sizes, hs, prec=1):
    specs = []
    for L, h in zip(sizes, hs):
        bonds, sub = lib.nqs_hypercube(L, 1)
        specs.append(dict(n_sites=L, n_hidden=2 * L, bonds=bonds, sublattice=sub, ham=lib.TFIM,
                          J=(1.0, 0.0), h=h, move=lib.MOVE_FLIP, is_complex=False, prec=prec))
    return lib.Batch(specs)


def test_batch_nonfinite_model_is_skipped(lib):
    """One model of a batch with a NaN local energy: the batch returns ENONFINITE in its
    info, that model's parameters are unchanged, the other models' updates equal a clean
    run's."""
    sizes, hs = [16, 24, 40], [0.7, 1.0, 1.3]
    b = _tfim_batch(lib, sizes, hs)
    nch, S = [64, 64, 64], 4
    ps = np.concatenate([synth.rbm_params(L, 2 * L, False, sigma=0.1, seed=80 + k)
                         for k, L in enumerate(sizes)]).astype(np.float32)
    chains = torch.empty(sum(c * L for c, L in zip(nch, sizes)), dtype=torch.int8, device=DEV)
    b.chain_init(chains, nch, seed=5)
    smp, el = b.sample(to_dev(ps), chains, nch, S, 4, seed=5, counter=0)
    ns = [c * S for c in nch]
    clean = to_dev(ps.copy())
    ic = b.sr_step(clean, smp, el, ns, lr=0.02, diag_shift=0.01, cg_tol=1e-8, cg_maxiter=60,
                   n_chains=nch)
    bad = el.clone()
    bad[ns[0] + 7] = float("nan")   # model 1
    for use_async in (False, True):
        pt = to_dev(ps.copy())
        if use_async:
            buf = b.sr_step_async(pt, smp, bad, ns, lr=0.02, diag_shift=0.01, cg_tol=1e-8,
                                  cg_maxiter=60, n_chains=nch)
            torch.cuda.synchronize()
            infos = lib.sr_infos_from_device(buf, 3)
        else:
            infos = b.sr_step(pt, smp, bad, ns, lr=0.02, diag_shift=0.01, cg_tol=1e-8,
                              cg_maxiter=60, n_chains=nch)
        assert [i["status"] for i in infos] == [ic[0]["status"], lib.ENONFINITE, ic[2]["status"]]
        off = np.cumsum([0] + b.n_params)
        got, ref = pt.cpu().numpy(), clean.cpu().numpy()
        assert np.array_equal(got[off[0]:off[1]], ref[off[0]:off[1]])
        assert np.array_equal(got[off[1]:off[2]].view(np.uint32), ps[off[1]:off[2]].view(np.uint32))
        assert np.array_equal(got[off[2]:off[3]], ref[off[2]:off[3]])


def test_batch_error_bars_match_oracle(lib):
    sizes, hs = [16, 30, 50], [0.6, 1.0, 1.4]
    b = _tfim_batch(lib, sizes, hs, prec=0)
    nch, S = [40, 64, 24], 6
    ps = np.concatenate([synth.rbm_params(L, 2 * L, False, sigma=0.1, seed=90 + k)
                         for k, L in enumerate(sizes)])
    chains = torch.empty(sum(c * L for c, L in zip(nch, sizes)), dtype=torch.int8, device=DEV)
    b.chain_init(chains, nch, seed=6)
    smp, el = b.sample(to_dev(ps), chains, nch, S, 4, seed=6, counter=0)
    ns = [c * S for c in nch]
    infos = b.sr_step(to_dev(ps.copy()), smp, el, ns, lr=0.02, diag_shift=0.01, cg_tol=1e-8,
                      cg_maxiter=60, n_chains=nch)
    e = el.cpu().numpy()
    off = 0
    for k in range(3):
        mean, var, err = osr.stats(e[off:off + ns[k]], n_chains=nch[k])
        assert abs(infos[k]["energy_re"] - mean) <= 1e-12 * abs(mean)
        assert abs(infos[k]["energy_err"] - err) <= 1e-9 * err, k
        off += ns[k]


def test_batch_step_graph_replays_match_direct_launches(lib):
    """Batched TFIM rings (uneven sizes, real FP32): sampling with the counter advanced on
    the device, local energies in the sweep, and the stream-ordered SR step, captured into
    one graph; every replay equals the same calls issued directly (chains, samples,
    energies, parameters and the information, bit for bit), and the random stream moves
    on from replay to replay."""
    sizes = [16, 34, 58, 90, 128]
    hs = [0.5, 0.8, 1.0, 1.2, 1.5]
    nch, S = [256] * len(sizes), 4
    ns = [c * S for c in nch]
    ps = np.concatenate([synth.rbm_params(L, 2 * L, False, sigma=0.05, seed=10 + k)
                         for k, L in enumerate(sizes)]).astype(np.float32)
    spins = sum(c * L for c, L in zip(nch, sizes))
    # one handle per side: a handle's job tables belong to the buffers of its last call,
    # and the captured graph reads the tables of its handle
    state = {}
    for tag in ("graph", "direct"):
        b = _tfim_batch(lib, sizes, hs)
        ch = torch.empty(spins, dtype=torch.int8, device=DEV)
        b.chain_init(ch, nch, seed=1234)
        state[tag] = dict(b=b, p=to_dev(ps.copy()), ch=ch,
                          smp=torch.empty(S * spins, dtype=torch.int8, device=DEV),
                          el=torch.empty(sum(ns), dtype=torch.float64, device=DEV),
                          cnt=torch.zeros(1, dtype=torch.int64, device=DEV),
                          ws=torch.empty(b.sr_workspace_bytes(ns), dtype=torch.uint8,
                                         device=DEV),
                          info=torch.zeros(len(sizes) * lib.SR_INFO_BYTES, dtype=torch.uint8,
                                           device=DEV))

    def step(st):
        st["b"].sample(st["p"], st["ch"], nch, S, 2, seed=1234, counter=0, samples=st["smp"],
                       eloc=st["el"], counter_dev=st["cnt"])
        st["b"].sr_step_async(st["p"], st["smp"], st["el"], ns, lr=0.02, diag_shift=0.01,
                              cg_tol=1e-6, cg_maxiter=40, workspace=st["ws"], n_chains=nch,
                              info=st["info"])

    # one uncaptured step on each side (uploads the job tables)
    step(state["graph"])
    step(state["direct"])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g, stream=s2):
            step(state["graph"])
    torch.cuda.synchronize()
    prev = None
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        step(state["direct"])
        torch.cuda.synchronize()
        G, D = state["graph"], state["direct"]
        for key in ("p", "ch", "smp", "el", "cnt", "info"):
            assert torch.equal(G[key], D[key]), (rep, key)
        assert int(G["cnt"].item()) == (rep + 2) * (S + 2)
        if prev is not None:
            assert not torch.equal(prev, G["smp"])
        prev = G["smp"].clone()
        infos = lib.sr_infos_from_device(G["info"], len(sizes))
        assert all(i["status"] in (lib.OK, lib.ENOTCONV) for i in infos)
