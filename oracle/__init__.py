"""FP64 CPU oracle for the VMC / RBM hot path of the NetKet paper (Carleo et al.,
"NetKet: A Machine Learning Toolkit for Many-Body Quantum Systems", 2019).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(``paper_1904_00031_amd``) never imports, links or calls anything here, and nothing
here imports the product path. The two share no code; the only common module is
``synth`` (seeded input generators, no arithmetic of the method).

Every function is a plain, slow, obviously-correct restatement of the definition it
cites, in float64 / complex128 numpy. Modules:

* ``lattice``      - hypercubic graphs with colored edges (Sec. 2.2.1).
* ``philox``       - Philox4x32-10 counter-based generator (Salmon et al., SC'11).
* ``rbm``          - RBM amplitude and its analytic log-derivatives (Sec. 2.2.2, 2.2.5).
* ``rbm_symm``     - the symmetric RBM (RbmSpinSymm, Sec. 2.2.2): filters shared over a
                     group of lattice symmetries.
* ``hamiltonian``  - TFIM / Heisenberg / J1-J2 connected elements and the local
                     energy of Eq. 5 (Sec. 2.2.1, 2.2.5).
* ``sampler``      - Metropolis chains on |psi|^2 (Eq. 4, Sec. 2.2.5).
* ``sr``           - statistics, force, stochastic reconfiguration and CG (Sec. 2.2.5,
                     Eq. 2).
* ``quant``        - bfloat16 rounding of the BF16 precision form.
* ``exact``        - exact diagonalisation, full enumeration, TFIM closed form and the
                     Bethe ansatz for the Heisenberg ring (ground truth for the pins).

Pinned status of each function is listed in the header of its module. Functions whose
result has no independent pin say "parity unpinned" there.
"""
