"""Plain, slow, CPU FP64 oracle of the DMRG3S hot path (Hubig, McCulloch,
Schollwoeck, Wolf, "A Strictly Single-Site DMRG Algorithm with Subspace
Expansion").

TEST INFRASTRUCTURE ONLY.  The product (the HIP library and its Python
binding) never imports, links or runs anything in this package; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark do.  The
oracle shares no code with the GPU path: it has its own MPO builders, its own
contractions (NumPy tensordot/einsum/SVD in float64), its own Lanczos and its
own sweep driver, each written from the paper.

Modules
  local_ops  spin-1/2 and spinful-fermion site operators
  mpo        MPO builders (exchange / hopping with Jordan-Wigner strings),
             the printed two-spin example MPO, MPO -> dense matrix
  ed         exact diagonalisation from bit strings / Fock states, built
             without any MPO (an independent check of the MPO builders)
  mps        left-canonicalisation (QR), state vector, norms
  contract   H_eff*psi, the explicit H_eff matrix, environment updates,
             expansion term, SVD truncation
  lanczos    Lanczos with full re-orthogonalisation
  dmrg3s     the sweep driver with the adaptive mixing factor
  adjoint    dE/dW of <psi|H_eff|psi>

Pins (see tests/test_oracle_*.py): the paper's worked two-spin example
(Sec. 4.3), closed forms (Heisenberg l=2,4; Hubbard dimer; free fermions;
Bethe-ansatz energy density), ED built without MPOs, Hermiticity, the energy
identity of Sec. 2, state invariance under expansion (Sec. 4.1),
variationality, and finite differences for the adjoint.
"""
