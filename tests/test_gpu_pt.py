"""GPU parity of parallel tempering (nqs_sample_pt, the samplers' tempering option of
Sec. 2.2.5) against oracle.sampler.sample_pt on the same random streams: the recorded
beta = 1 samples bit-exact (a chain may part from the oracle only after a near-tie of one
of its proposals or exchanges, recorded by the oracle), and when no chain parts, every
replica's configuration, the temperature indices and the exchange counts too."""
import numpy as np
import pytest
import torch

import cases
from oracle import hamiltonian as oh, sampler as osamp

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def start(m, om, C, R, seed, shuffle):
    """Replica configurations from nqs_chain_init and temperature indices, either in
    replica order or a seeded permutation per chain."""
    ch = torch.empty((C * R, om.n_sites), dtype=torch.int8, device=DEV)
    m.chain_init(ch, seed=seed)
    reps = ch.view(C, R, om.n_sites)
    if shuffle:
        rng = np.random.default_rng(seed)
        tix = np.stack([rng.permutation(R) for _ in range(C)]).astype(np.int32)
    else:
        tix = np.tile(np.arange(R, dtype=np.int32), (C, 1))
    return reps, to_dev(tix)


@pytest.mark.parametrize("name,R,margin", [
    ("tfim10_real_f64", 2, 1e-12), ("heis40_cplx_f64", 3, 1e-12), ("j1j2_4x4_cplx_f64", 4, 1e-12),
    ("tfim37_cplx_f64", 4, 1e-12), ("j1j2_6x6_cplx_f64", 2, 1e-12), ("heis12_real_f64_flip", 3, 1e-12),
    ("heis40_cplx_f32", 4, 1e-4), ("tfim37_real_f32", 3, 1e-4), ("heis6x6_cplx_f32", 2, 1e-4),
    ("tfim300_cplx_f32_m150", 2, 1e-4)])
def test_pt_matches_oracle(lib, name, R, margin):
    m, om = cases.build(lib, name)
    p = cases.params(name, seed=29)
    C, S, D = 12, 5, 2
    reps, tix = start(m, om, C, R, seed=77, shuffle=(R > 2))
    init, tix0 = reps.cpu().numpy().copy(), tix.cpu().numpy().copy()
    nacc = torch.zeros(C * R, dtype=torch.int64, device=DEV)
    nsw = torch.zeros(C, dtype=torch.int64, device=DEV)
    smp, el = m.sample_pt(to_dev(p), reps, tix, S, D, seed=4321, counter=11, chain_offset=3,
                          n_accepted=nacc, n_swaps=nsw, with_eloc=True)
    ties = []
    exp, last, tix_o, nsw_o = osamp.sample_pt(om, cases.oracle_params(name, p), init, tix0, S, D,
                                              seed=4321, counter=11, chain_offset=3,
                                              record_ties=ties, tie_margin=margin)
    got = smp.cpu().numpy()
    diverged = cases.compare_chains(got, exp, ties, D)
    if diverged == 0:
        assert np.array_equal(reps.cpu().numpy(), last)
        assert np.array_equal(tix.cpu().numpy(), tix_o)
        assert np.array_equal(nsw.cpu().numpy(), nsw_o)
    # the temperatures of each chain stay a permutation; counts within their bounds
    t = tix.cpu().numpy()
    assert np.array_equal(np.sort(t, axis=1), np.tile(np.arange(R), (C, 1)))
    assert np.all((nsw.cpu().numpy() >= 0) & (nsw.cpu().numpy() <= (S + D) * (R - 1)))
    assert np.all((nacc.cpu().numpy() >= 0) & (nacc.cpu().numpy() <= (S + D) * om.n_sites))
    # local energies of the recorded samples
    ee = oh.local_energy(om, cases.oracle_params(name, p), got.reshape(-1, om.n_sites))
    assert np.abs(el.cpu().numpy() - ee).max() <= cases.tol(name) * max(1.0, np.abs(ee).max())


def test_pt_exchanges_happen_and_resume_is_bit_exact(lib):
    """Two calls (counter advanced, replicas and temperatures carried) equal one call; at
    these amplitudes the exchanges are accepted often."""
    name = "heis40_cplx_f64"
    m, om = cases.build(lib, name)
    p = to_dev(cases.params(name, seed=3))
    C, R = 16, 4
    reps1, tix1 = start(m, om, C, R, seed=8, shuffle=True)
    reps2, tix2 = reps1.clone(), tix1.clone()
    nsw = torch.zeros(C, dtype=torch.int64, device=DEV)
    a, _ = m.sample_pt(p, reps1, tix1, 6, 0, seed=5, counter=100, n_swaps=nsw)
    b1, _ = m.sample_pt(p, reps2, tix2, 3, 0, seed=5, counter=100)
    b2, _ = m.sample_pt(p, reps2, tix2, 3, 0, seed=5, counter=103)
    assert torch.equal(a, torch.cat([b1, b2]))
    assert torch.equal(reps1, reps2) and torch.equal(tix1, tix2)
    assert int(nsw.sum()) > C


def test_pt_rejects_what_it_does_not_run(lib):
    m, om = cases.build(lib, "heis40_cplx_f32")
    p = to_dev(cases.params("heis40_cplx_f32"))
    for R in (5, 1):
        reps = torch.zeros((4, R, om.n_sites), dtype=torch.int8, device=DEV)
        tix = torch.zeros((4, R), dtype=torch.int32, device=DEV)
        with pytest.raises(lib.NQSError) as ex:
            m.sample_pt(p, reps, tix, 2, 0, seed=1, counter=0)
        assert ex.value.status == lib.EINVAL
    # the wide FP32 sweep (more than 256 hidden units, tables beyond LDS) does not temper
    m, om = cases.build(lib, "heis4x4_cplx_f32_m1024")
    p = to_dev(cases.params("heis4x4_cplx_f32_m1024"))
    reps = torch.ones((4, 2, om.n_sites), dtype=torch.int8, device=DEV)
    tix = torch.zeros((4, 2), dtype=torch.int32, device=DEV)
    with pytest.raises(lib.NQSError) as ex:
        m.sample_pt(p, reps, tix, 2, 0, seed=1, counter=0)
    assert ex.value.status == lib.EUNSUPPORTED
