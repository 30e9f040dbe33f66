"""Oracle: exact ground truth for small systems (test infrastructure only).

Sec. 2.1 lists exact diagonalisation among the toolkit's tools (used to check variational
results); here it pins the oracle itself:

* ``dense_hamiltonian`` / ``sparse_hamiltonian``: H assembled from Kronecker products of
  Pauli matrices, with no reference to the connected-element code of ``hamiltonian``.
  Basis order: site 0 is the leftmost Kronecker factor (most significant bit); bit value 0
  is spin up (sz = +1).
* ``marshall_unitary``: the diagonal U = prod_{i in sublattice 1} sz_i.
* ``exact_energy``: <psi|H|psi>/<psi|psi> by full enumeration.
* ``ground_state``: the lowest eigenvector (targets of the supervised loss).
* ``tfim_ground_energy``: free-fermion closed form of the periodic TFIM ring.
* ``heisenberg_ring_bethe``: Bethe-ansatz ground energy of the periodic Heisenberg ring.

Pins (tests/test_oracle_exact.py): closed form and Bethe ansatz against sparse ED of the
Kronecker-built H (N = 9..16 and N = 16, 20), ED against published exact-diagonalisation
energies of the 4x4 Heisenberg and J1-J2 lattices (tests/golden/reference_energies.txt,
with their sources).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import lattice, rbm

SX = np.array([[0.0, 1.0], [1.0, 0.0]])
SY = np.array([[0.0, -1j], [1j, 0.0]])
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])
ID = np.eye(2)


def _site_op(op, i, n):
    mats = [sp.identity(2 ** i, format="csr"), sp.csr_matrix(op), sp.identity(2 ** (n - i - 1), format="csr")]
    return sp.kron(sp.kron(mats[0], mats[1]), mats[2], format="csr")


def sparse_hamiltonian(model):
    n = model.n_sites
    dim = 2 ** n
    H = sp.csr_matrix((dim, dim), dtype=np.complex128)
    z = [_site_op(SZ, i, n) for i in range(n)]
    x = [_site_op(SX, i, n) for i in range(n)]
    if model.ham == 0:
        for c, bl in enumerate(model.bonds):
            for i, j in bl:
                H = H - model.J[c] * (z[i] @ z[j])
        for i in range(n):
            H = H - model.h * x[i]
    else:
        y = [_site_op(SY, i, n) for i in range(n)]
        for c, bl in enumerate(model.bonds):
            for i, j in bl:
                H = H + model.J[c] * (x[i] @ x[j] + y[i] @ y[j] + z[i] @ z[j])
    if model.marshall:
        U = marshall_unitary(model)
        H = U @ H @ U.conj().T
    return H.tocsr()


def dense_hamiltonian(model):
    return sparse_hamiltonian(model).toarray()


def marshall_unitary(model):
    n = model.n_sites
    U = sp.identity(2 ** n, format="csr", dtype=np.complex128)
    for i in range(n):
        if model.sublattice[i]:
            U = U @ _site_op(SZ, i, n)
    return U


def exact_energy(model, params, machine=None):
    """<psi|H|psi>/<psi|psi> over all 2**N basis states (Sec. 2.2.5 first line of Eq. 5)."""
    confs = lattice.all_configs(model.n_sites)
    lp = (rbm.log_psi(params, confs, model.n_sites, model.n_hidden) if machine is None
          else machine.log_psi(params, confs))
    psi = np.exp(lp - np.max(lp.real))
    H = sparse_hamiltonian(model)
    return (np.vdot(psi, H @ psi) / np.vdot(psi, psi))


def exact_probabilities(model, params):
    """pi(sigma) of Eq. 4 over all basis states (same order as lattice.all_configs)."""
    confs = lattice.all_configs(model.n_sites)
    lp = rbm.log_psi(params, confs, model.n_sites, model.n_hidden)
    w = np.exp(2.0 * (lp.real - lp.real.max()))
    return confs, w / w.sum()


def sz_sector_indices(n, total=0):
    confs = lattice.all_configs(n)
    return np.nonzero(confs.sum(axis=1) == total)[0]


def ground_energy(model, sector_sz=None, k=1):
    """Lowest eigenvalue(s) of the Kronecker-built H, optionally restricted to a total-Sz
    sector (H conserves total Sz for the Heisenberg models)."""
    H = sparse_hamiltonian(model)
    if sector_sz is not None:
        idx = sz_sector_indices(model.n_sites, sector_sz)
        H = H[idx][:, idx]
    if H.shape[0] <= 2048:
        return np.linalg.eigvalsh(H.toarray())[:k]
    vals = spla.eigsh(H, k=k, which="SA", tol=1e-12)[0]
    return np.sort(vals)


def ground_state(model):
    """Lowest eigenvalue and eigenvector of the Kronecker-built H over all 2**N basis states
    (lattice.all_configs order), with the phase fixed so that its largest component is real
    and positive."""
    H = sparse_hamiltonian(model)
    if H.shape[0] <= 2048:
        vals, vecs = np.linalg.eigh(H.toarray())
    else:
        vals, vecs = spla.eigsh(H, k=1, which="SA", tol=1e-13)
    v = vecs[:, np.argmin(vals)]
    k = np.argmax(np.abs(v))
    return float(np.min(vals)), v * (np.conj(v[k]) / abs(v[k]))


def tfim_ground_energy(n, J=1.0, h=1.0):
    """Periodic ferromagnetic TFIM ring: -sum_m sqrt(J^2 + h^2 - 2 J h cos k_m),
    k_m = (2m+1) pi / n (Jordan-Wigner free fermions, even-parity sector)."""
    m = np.arange(n)
    k = (2 * m + 1) * np.pi / n
    return -np.sum(np.sqrt(J * J + h * h - 2 * J * h * np.cos(k)))


def heisenberg_ring_bethe(n, J=1.0, iters=200000, tol=1e-15):
    """Ground energy (Pauli units) of the periodic spin-1/2 Heisenberg antiferromagnet
    ring with even n, from the logarithmic Bethe equations
        n * arctan(2 lam_a) = pi I_a + sum_b arctan(lam_a - lam_b),
    I_a = -(M-1)/2 .. (M-1)/2 for M = n/2 magnons, energy in spin units
        E_S = J n / 4 - sum_a 2 J / (1 + 4 lam_a^2),
    and E_Pauli = 4 E_S. Solved by damped fixed-point iteration."""
    if n % 2:
        raise ValueError("even ring length required")
    M = n // 2
    I = np.arange(M) - (M - 1) / 2.0
    lam = 0.5 * np.tan(np.pi * I / n)
    for _ in range(iters):
        rhs = (np.pi * I + np.arctan(lam[:, None] - lam[None, :]).sum(axis=1)) / n
        new = 0.5 * np.tan(rhs)
        if np.max(np.abs(new - lam)) < tol:
            lam = new
            break
        lam = 0.5 * lam + 0.5 * new
    es = J * n / 4.0 - np.sum(2.0 * J / (1.0 + 4.0 * lam ** 2))
    return 4.0 * es
