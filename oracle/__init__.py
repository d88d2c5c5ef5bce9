"""FP64 CPU oracle for the local-global solver with frictional contact.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP solver; the two
meet only at the seeded scene generator (``paper_2503_15078_amd.scenes``),
which builds inputs and holds none of the method's arithmetic.

The oracle follows the paper step by step, in float64, with the global step
done by a direct sparse factorisation of the system matrix (the plain
definition u = A^-1 b) instead of the sparse inverse S, and with the Delassus
operator W = H A^-1 H^T formed by direct multi-right-hand-side solves.

Modules
  fem            rest quantities, lumped mass, PD weights, system matrix  (Sec. 3.3, Eq. PD global)
  material       energies on signed singular values and the local prox     (Eq. PD local)
  contact        obstacle distances, contact frames, Fischer-Burmeister    (App. A, App. B)
  cr             Conjugate Residual                                        (Sec. 6, constraint solver)
  sparse_inverse elimination tree and L^-1 on small matrices               (Sec. 4.2, Theorem 1)
  sim            the frame / iteration loop of Algorithm 4
  brute_ncp      brute-force solutions of small contact problems (pins only)
  selfcontact    surface triangles, vertex-triangle self-contacts, multi-node rows
                 and their Delassus block                                 (Sec. 6, Sec. 3.2, App. A)

Pinning status of each function is stated in its docstring; functions with
no independent pin say "parity unpinned".
"""
