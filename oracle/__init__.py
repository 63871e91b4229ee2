"""CPU FP64 oracle for HIF-IE (Ho & Ying, "Hierarchical interpolative
factorization for elliptic operators: integral equations", arXiv 1307.2666).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything under ``oracle/``: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is a plain, slow, obviously correct NumPy/SciPy implementation:

* ``kernels``    -- the discretized operator ``A = diag(a) + diag(b) K diag(c)``
                    of eqn (1.1) under piecewise-constant collocation
                    (Section 3.1, eqn kernel-integral), closed-form self terms,
                    dense assembly, exact matvec.
* ``tree``       -- uniform quadtree/octree depth, the cell / face / edge
                    partitions of Algorithms 4.1 and 4.2, proxy surfaces
                    (Section 3.3).
* ``idqr``       -- interpolative decomposition by column-pivoted QR
                    (Lemma 2.2) with the adaptive rank rule of Section 2.2.
* ``factor``     -- recursive skeletonization factorization (Algorithm 3.1)
                    and HIF-IE (Algorithms 4.1 / 4.2) with accelerated
                    compression (Sections 3.3, 4.3) and the second-kind
                    modification (Section 4.4), followed by the factored
                    apply / solve sweeps of eqns (rskelf), (hifie2), (hifie3).
* ``estimators`` -- power-iteration error estimates e_a, e_s and
                    right-preconditioned GMRES (Section 5).

Every function cites the passage of the paper it follows; where the paper is
silent or ambiguous, the docstring states the reading taken.
"""
