"""Oracle: lattice spin Hamiltonians and the local energy of Eq. 5 (test infrastructure only).

Sec. 2.2.1 provides the transverse-field Ising and Heisenberg models on a graph, with
edge colors selecting the bond type (GraphOperator: 2-local bond terms per color plus
1-local site terms). Operators are Pauli matrices (the paper fixes no normalisation;
Pauli units are 4x the spin-1/2 ones).

* TFIM:        H = - sum_c J_c sum_{(i,j) in color c} sz_i sz_j - h sum_i sx_i
               (ferromagnetic sign; identical spectrum to the antiferromagnet for
               bipartite lattices).
* Heisenberg:  H = sum_c J_c sum_{(i,j) in color c} (sx_i sx_j + sy_i sy_j + sz_i sz_j).
               sx sx + sy sy maps |up,down> <-> |down,up> with element 2.
* Marshall rotation (optional): H' = U H U^dagger with U = prod_{i in sublattice 1} sz_i.
               Only the off-diagonal exchange element of bonds joining the two
               sublattices changes sign.

Eq. 5, Sec. 2.2.5: E_loc(sigma) = sum_sigma' <sigma|H|sigma'> psi(sigma')/psi(sigma), and
<H> is its average over sigma ~ |psi|^2 (Eq. 4).

Pins (tests/test_oracle_hamiltonian.py): the exact identity
sum_sigma pi(sigma) E_loc(sigma) = <psi|H|psi>/<psi|psi> with H assembled independently
from Kronecker products of Pauli matrices (``exact.dense_hamiltonian``), for every model
and with/without the Marshall rotation; the special cases psi = const (E_loc is the row
sum of H) and J=0 TFIM (uniform psi is an eigenstate, zero variance).
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import rbm

TFIM = 0
HEISENBERG = 1
MOVE_FLIP = 0
MOVE_EXCHANGE = 1


@dataclass
class Model:
    n_sites: int
    n_hidden: int
    bonds: List[np.ndarray]                 # per color: int [B_c, 2]
    ham: int = TFIM
    J: tuple = (1.0, 0.0)
    h: float = 1.0
    marshall: bool = False
    sublattice: Optional[np.ndarray] = None
    move: int = MOVE_FLIP
    is_complex: bool = False

    @property
    def n_params(self):
        return rbm.n_params(self.n_sites, self.n_hidden)


def bond_sign(model, color, i, j):
    """Marshall sign of the exchange element on bond (i, j): -1 when the rotation is on
    and the bond joins the two sublattices, else +1."""
    if model.marshall and model.sublattice[i] != model.sublattice[j]:
        return -1.0
    return 1.0


def connected(model, sigma):
    """Return (diag, list of (sigma', element)) for one configuration sigma [N]."""
    s = np.asarray(sigma, dtype=np.int64)
    diag = 0.0
    off = []
    if model.ham == TFIM:
        for c, bl in enumerate(model.bonds):
            for i, j in bl:
                diag += -model.J[c] * s[i] * s[j]
        if model.h != 0.0:
            for i in range(model.n_sites):
                sp = s.copy()
                sp[i] = -sp[i]
                off.append((sp, -model.h))
    elif model.ham == HEISENBERG:
        for c, bl in enumerate(model.bonds):
            if model.J[c] == 0.0:
                continue
            for i, j in bl:
                diag += model.J[c] * s[i] * s[j]
                if s[i] != s[j]:
                    sp = s.copy()
                    sp[i], sp[j] = s[j], s[i]
                    off.append((sp, 2.0 * model.J[c] * bond_sign(model, c, i, j)))
    else:
        raise ValueError("unknown Hamiltonian")
    return diag, off


def local_energy(model, params, sigma, machine=None):
    """E_loc for each row of sigma [n, N] (Eq. 5), ratios from log psi differences.
    machine: any ansatz with log_psi(params, sigma) (default: the RBM of the model)."""
    sig = np.atleast_2d(np.asarray(sigma))
    if machine is None:
        def log_psi(p, s):
            return rbm.log_psi(p, s, model.n_sites, model.n_hidden)
    else:
        log_psi = machine.log_psi
    lp = log_psi(params, sig)
    out = np.zeros(sig.shape[0], dtype=np.complex128)
    for k in range(sig.shape[0]):
        diag, off = connected(model, sig[k])
        e = complex(diag)
        if off:
            sps = np.array([sp for sp, _ in off])
            els = np.array([el for _, el in off])
            lpp = log_psi(params, sps)
            e += np.sum(els * np.exp(lpp - lp[k]))
        out[k] = e
    if not model.is_complex and not np.iscomplexobj(params):
        return out.real.copy()
    return out
