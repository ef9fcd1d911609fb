"""CPU FP64 oracle for the GenEO-preconditioned CG solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (the HIP library and its Python binding) never
calls it, and it shares no code with that path: it only consumes the seeded
inputs built by :mod:`workloads`.

It is plain and slow on purpose: every function follows one definition of the
paper (Butler et al., arXiv 1901.05188) and cites the passage it restates.

* :mod:`oracle.fem`   -- Sections 2 (eq-strain, eq-hooke, eq-fe,
  eqn:fe_matrix_system) and 6 (eq-fe-darcy): Q1 element integrals, material
  tensors, assembly with Dirichlet DOFs eliminated.
* :mod:`oracle.dd`    -- Section 3.1 (overlapping subdomains, V_{h,0}) and
  Section 3.2 (Definition of the subdomain overlap, Definition of the
  partition of unity, Section 3.3.1 standard PoU).
* :mod:`oracle.geneo` -- Section 3.2 eq-geneo and the GenEO coarse space
  definition, Section 3.3.2 eqm:matrixForm, Section 3.3.3 coarse matrix.
* :mod:`oracle.pcg`   -- Section 3.1 (CG, eqn:onelevelAS, two-level AS).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants or brute force; see the pin list in each
module docstring.
"""
