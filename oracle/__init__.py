"""CPU FP64 oracle for the ACSE residual hot path (arXiv 2604.02550).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything under this package.  It
is used by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.

The oracle shares no code with the GPU path.  It is written from the paper in
the plainest form available:

* ``fermion``  -- brute force in the full Fock space (Jordan-Wigner matrices):
  Hamiltonian of Eq. (1), exact FCI, exact 1-/2-/3-RDMs of Eq. (6), and the
  commutator expectations of Eq. (4) and Eq. (9).  This is the pin for
  everything else.
* ``rdm``      -- spin-orbital tensors built from spatial inputs: the reduced
  Hamiltonian of Eq. (2), the spin blocks and traces of App. A, the cumulant
  expansion of Eq. (7) and the Valdemoro 3-RDM of App. C, Eq. (C5).
* ``residual`` -- the residual map of Eq. (4)/(5) (tier A, materialised 3-RDM,
  small r), the factorised form of App. D.1, Eqs. (D2)-(D4) with the
  transposition forms of App. B, Eqs. (B8)-(B9) (tier B, any r, 3-RDM never
  formed), and a single-element evaluator for sampled checks at large r.
* ``step``     -- the Euler update of Eq. (9), the active-active mask, trace
  restoration, the 1-RDM contraction and the energy Tr(K 2D).
* ``adjoint``  -- vector-Jacobian products of the residual and the energy by
  reverse-mode differentiation of the tier-B torch forward, projected onto
  the symmetry subspaces of the inputs.

All arithmetic is float64.  Readings of the paper where it is silent, garbled
or self-inconsistent are stated in the docstrings where they are used.
"""
