"""Writes ed_energies.json from the CPU reference only (exact diagonalisation).

Run from the repository root:  python tests/golden/make_golden.py
Every value is a ground energy of a physical Hamiltonian built spin by spin
from its textbook definition (oracle.physics_ref), by sparse Lanczos.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import physics_ref as P  # noqa: E402


def main():
    out = {
        "_source": "tests/golden/make_golden.py (oracle.physics_ref, scipy eigsh, tol 1e-14)",
        "tfim_chain_L16_h1": P.ground_energy(P.tfim_chain_hamiltonian(16, 1.0)),
        "tfim_chain_L8_h1": P.ground_energy(P.tfim_chain_hamiltonian(8, 1.0)),
        "xxx_chain_L16": P.ground_energy(P.heisenberg_chain_hamiltonian(16)),
        "xxx_chain_L8": P.ground_energy(P.heisenberg_chain_hamiltonian(8)),
        "torus_tfim_4x4_h3": P.ground_energy(P.torus_tfim_hamiltonian(4, 4, 3.0)),
        "torus_tfim_4x3_h3": P.ground_energy(P.torus_tfim_hamiltonian(4, 3, 3.0)),
    }
    with open(os.path.join(HERE, "ed_energies.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
