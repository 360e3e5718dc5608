#!/usr/bin/env python3
"""Writes the stored reference values of tests/golden/ from the oracle only
(exact diagonalisation and closed forms of oracle/exact.py).  Run from the
repository root:  python tests/golden/make_golden.py

Every value is a property of a Hamiltonian, not of DMRG:
- open Heisenberg chains (the model of Sec. III without the Q term), ground
  energy by sparse exact diagonalisation in the S^z = 0 sector;
- open XX chain: free fermions, E0 = sum over negative single-particle
  energies J cos(k pi / (N + 1));
- open transverse-field Ising chain (Pauli matrices): E0 = -sum of the
  singular values of the bidiagonal matrix with h on the diagonal and J
  above it, and dE0/dh from first-order perturbation of those values.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact, models  # noqa: E402


def main():
    out = {}
    for N in (10, 12, 16):
        e = exact.ground_state(models.heisenberg_terms(models.chain_bonds(N)), N, 0)[0][0]
        out["heisenberg_chain_N%d_J1_E0" % N] = float(e)
    for N in (10, 16, 32):
        out["xx_chain_N%d_J1_E0" % N] = float(exact.xx_chain_energy(N, 1.0))
    for N, h in ((10, 0.8), (16, 0.7)):
        out["tfim_chain_N%d_J1_h%g_E0" % (N, h)] = float(exact.tfim_chain_energy(N, 1.0, h))
        out["tfim_chain_N%d_J1_h%g_dE0dh" % (N, h)] = float(exact.tfim_chain_dE_dh(N, 1.0, h))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_energies.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(path)


if __name__ == "__main__":
    main()
