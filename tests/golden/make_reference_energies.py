"""Writes the computed lines of reference_energies.txt from the oracle alone:

    python tests/golden/make_reference_energies.py

The free-fermion TFIM closed form and the Bethe-ansatz ring energies come from
``oracle.exact``; the literature exact-diagonalisation lines (4x4 lattices) are kept as
published, with their source. Values are printed with 17 significant digits."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "reference_energies.txt")

LITERATURE = """# 4x4 periodic Heisenberg antiferromagnet: E/N = -0.7017802 in spin-1/2 units
# (exact diagonalisation, e.g. Schulz, Ziman, Poilblanc, J. Phys. I 6, 675 (1996)).
heis_4x4_per_site_spin_units -0.7017802 literature-ED
# 4x4 periodic J1-J2 at J2/J1 = 0.5: E/N = -0.5286 in spin-1/2 units (same reference).
j1j2_4x4_j2_0.5_per_site_spin_units -0.5286 literature-ED
"""


def main():
    lines = ["# Exact ground energies used as pins, Pauli units (4x the spin-1/2 convention), J1 = 1.",
             "# Each line: name value source. Lines marked closed-form / bethe-ansatz are written",
             "# by make_reference_energies.py from the oracle.",
             "# TFIM ring, N=10, h=1, periodic: free-fermion closed form -2/sin(pi/20) (Pfeuty 1970).",
             "tfim_n10_h1 %.17g closed-form" % exact.tfim_ground_energy(10, 1.0, 1.0),
             "# Heisenberg ring, periodic, N=20 (the paper's worked VMC example) and N=40:",
             "# logarithmic Bethe equations solved numerically.",
             "heis_ring_n20 %.17g bethe-ansatz" % exact.heisenberg_ring_bethe(20),
             "heis_ring_n40 %.17g bethe-ansatz" % exact.heisenberg_ring_bethe(40)]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n" + LITERATURE)


if __name__ == "__main__":
    main()
