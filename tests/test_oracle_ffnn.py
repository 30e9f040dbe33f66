"""Pins of the FFNN oracle (Sec. 2.2.2: dense layers with ln cosh / tanh activations)
against what the paper and the mathematics fix: the RBM without visible bias as the one
ln cosh layer, the composition limit of a small first tanh layer, finite differences,
the parity symmetry, and the dense Hamiltonian."""
import numpy as np
import pytest

from oracle import exact, ffnn, hamiltonian as oh, lattice, rbm


def rand_params(net, rng, s, cplx):
    p = rng.normal(0, s, net.n_params)
    if cplx:
        p = p + 1j * rng.normal(0, s, net.n_params)
    return p


def spins(rng, n, N):
    return rng.choice(np.array([-1, 1], dtype=np.int8), size=(n, N))


@pytest.mark.parametrize("cplx", [False, True])
def test_one_lncosh_layer_is_the_rbm_without_visible_bias(cplx):
    rng = np.random.default_rng(1)
    N, M = 7, 9
    net = ffnn.FFNN(N, [M], [ffnn.LNCOSH])
    p = rand_params(net, rng, 0.5, cplx)
    (b, W), = net.unpack(p)
    pr = rbm.pack(np.zeros(N, dtype=p.dtype), b, W)
    s = spins(rng, 40, N)
    assert np.abs(net.log_psi(p, s) - rbm.log_psi(pr, s, N, M)).max() <= 1e-13
    O = net.log_derivatives(p, s)
    Or = rbm.log_derivatives(pr, s, N, M)
    assert np.abs(O - Or[:, N:]).max() <= 1e-13


def test_small_tanh_layer_composes_into_the_rbm():
    """tanh(eps x) = eps x + O(eps^3): a first tanh layer (width K) of weights eps A, bias
    eps c followed by an ln cosh layer (W, b) is the RBM with weights eps W A and bias
    b + eps W c, up to |W| |eps x|^3 / 3 in the angles."""
    rng = np.random.default_rng(2)
    N, K, M, eps = 6, 5, 4, 1e-4
    net = ffnn.FFNN(N, [K, M], [ffnn.TANH, ffnn.LNCOSH])
    A = rng.normal(0, 1, (K, N)) + 1j * rng.normal(0, 1, (K, N))
    c = rng.normal(0, 1, K) + 1j * rng.normal(0, 1, K)
    W = rng.normal(0, 1, (M, K)) + 1j * rng.normal(0, 1, (M, K))
    b = rng.normal(0, 1, M) + 1j * rng.normal(0, 1, M)
    p = net.pack([(eps * c, eps * A), (b, W)])
    pr = rbm.pack(np.zeros(N, dtype=np.complex128), b + eps * W @ c, eps * W @ A)
    s = spins(rng, 30, N)
    x = np.abs(c)[None, :] + np.abs(s @ np.abs(A).T)
    bound = (np.abs(W).sum(axis=1).max() * (eps * x.max()) ** 3) * M
    assert np.abs(net.log_psi(p, s) - rbm.log_psi(pr, s, N, M)).max() <= 10 * bound + 1e-14
    # a second layer with its columns permuted does not (the pin sees how W meets z_1)
    p_bad = net.pack([(eps * c, eps * A), (b, W[:, ::-1])])
    assert np.abs(net.log_psi(p_bad, s) - rbm.log_psi(pr, s, N, M)).max() > 1e3 * bound


@pytest.mark.parametrize("sizes,acts", [([6, 5], [ffnn.TANH, ffnn.LNCOSH]),
                                        ([8, 4, 3], [ffnn.LNCOSH, ffnn.TANH, ffnn.LNCOSH]),
                                        ([5, 5], [ffnn.LNCOSH, ffnn.TANH])])
def test_log_derivatives_are_finite_differences(sizes, acts):
    """Holomorphic central differences, eps = 1e-6, over every parameter."""
    rng = np.random.default_rng(3)
    N = 5
    net = ffnn.FFNN(N, sizes, acts)
    p = rand_params(net, rng, 0.4, True)
    s = spins(rng, 6, N)
    O = net.log_derivatives(p, s)
    eps = 1e-6
    for k in range(net.n_params):
        e = np.zeros(net.n_params, dtype=np.complex128)
        e[k] = eps
        fd = (net.log_psi(p + e, s) - net.log_psi(p - e, s)) / (2 * eps)
        assert np.abs(fd - O[:, k]).max() <= 1e-7 * max(1.0, np.abs(O).max()), k


def test_zero_biases_and_lncosh_last_give_an_even_amplitude():
    rng = np.random.default_rng(4)
    N = 8
    net = ffnn.FFNN(N, [6, 7], [ffnn.TANH, ffnn.LNCOSH])
    layers = [(np.zeros(6, dtype=complex), rng.normal(0, 0.5, (6, N)) + 0.3j),
              (np.zeros(7, dtype=complex), rng.normal(0, 0.5, (7, 6)) - 0.2j)]
    p = net.pack(layers)
    s = spins(rng, 20, N)
    assert np.abs(net.log_psi(p, s) - net.log_psi(p, -s)).max() <= 1e-13
    # with biases the symmetry is broken
    layers[1] = (np.full(7, 0.3 + 0.1j), layers[1][1])
    p = net.pack(layers)
    assert np.abs(net.log_psi(p, s) - net.log_psi(p, -s)).max() > 1e-3


@pytest.mark.parametrize("ham,move", [(0, 0), (1, 1)])
def test_local_energy_of_the_network_against_the_dense_hamiltonian(ham, move):
    rng = np.random.default_rng(5)
    N = 8
    bonds, sub = lattice.hypercube(N, 1)
    om = oh.Model(N, 1, bonds, ham=ham, J=(1.0, 0.0), h=0.8, marshall=ham == 1,
                  sublattice=sub, move=move, is_complex=True)
    net = ffnn.FFNN(N, [10, 6], [ffnn.LNCOSH, ffnn.TANH])
    p = rand_params(net, rng, 0.3, True)
    confs = lattice.all_configs(N)
    if ham == 1:
        confs = confs[confs.sum(axis=1) == 0]
    el = oh.local_energy(om, p, confs, machine=net)
    lp = net.log_psi(p, confs)
    w = np.exp(2 * (lp.real - lp.real.max()))
    E = np.sum(w * el) / w.sum()
    Eex = exact.exact_energy(om, p, machine=net) if ham == 0 else None
    if ham == 0:
        assert abs(E - Eex) <= 1e-12 * abs(Eex)
    else:
        # Heisenberg conserves Sz: the sector sum equals <psi P|H|P psi> / <psi P|P psi>
        H = exact.sparse_hamiltonian(om)
        idx = exact.sz_sector_indices(N, 0)
        allc = lattice.all_configs(N)
        lpa = net.log_psi(p, allc)
        psi = np.zeros(2 ** N, dtype=np.complex128)
        psi[idx] = np.exp(lpa[idx] - lpa[idx].real.max())
        Eex = np.vdot(psi, H @ psi) / np.vdot(psi, psi)
        assert abs(E - Eex) <= 1e-12 * abs(Eex)
