"""CPU float64 reference for the binary-TTN energy-minimisation sweep.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import, call or execute anything in this
package.  The GPU library never does, and this package never imports the GPU
library: the two share no code.  Inputs reach both sides from the seeded
generators in ``paper_1905_01331_amd.inputs`` (pure numpy, none of the
method's arithmetic).

Modules
-------
ttn_ref         the sweep, written from Secs. II.C and III of the paper
ttn_positional  the same with an isometry of its own at every node
ttn_complex     the same for complex tensors (Hamiltonians with complex
                matrix elements): bra copies conjugated
physics_ref     exact diagonalisation, closed forms and brute-force state
                vectors used to pin the three against mathematics other than
                themselves

Every function in them has at least one pin in ``tests/`` (see the module
docstrings).  Nothing here is parity-unpinned.
"""
