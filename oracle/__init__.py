"""CPU FP64 oracle for real-space parallel DMRG (Stoudenmire & White,
"Real-Space Parallel Density Matrix Renormalization Group").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised reference written from the paper.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path (the HIP library and its Python binding) never does, and the
two share no code.  Inputs common to both sides come from the seeded
generators in ``paper_1301_3494_amd.synth``, which hold no DMRG arithmetic.

Modules
-------
models    lattices and Hamiltonian term lists (Sec. III)
mpo       finite-state-machine MPO builder, dense contraction, Schmidt ranks
exact     exact diagonalisation and free-fermion closed forms (test pins)
blocks    U(1) block-sparse bonds and tensors
dmrg      environments, two-site H_eff, Davidson / Lanczos, truncated SVD with
          the Appendix recursion, split / merge (Eqs. eqn:inverse, eqn:isvd,
          eqn:merge), serial and real-space parallel sweeps (Sec. II, Fig. 4)
grad      Hellmann-Feynman gradients dE/dW and finite-difference driver
gauge     inverse canonical gauge (Sec. IV) and local measurements from the
          orthogonality centres

Parity status of each function is stated in its docstring; everything here
is pinned by the ``-m "not gpu"`` tests against exact diagonalisation,
closed forms, dense constructions or invariants, except where a docstring
says "parity unpinned".
"""
