"""CPU oracle for the QTT finite-element elasticity solve (test infrastructure only).

This package is the slow, plainly written FP64 reference that the GPU library is
checked against.  It is imported only by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; the product path never calls it
and shares no code with it.

Modules
-------
fem    O1: element-by-element sparse Q1 assembly of the Galerkin system of
       Sec. 3 (eq. finbilform / femsys, elassembly, grads) for the isotropic law
       of Sec. 2, consistent mass loads f = M f0 (Sec. 5.3), Dirichlet/Neumann
       faces, and a sparse direct solve.
tt     tensor-train (MPS / MPO) primitives of Sec. 4: QTT folding (the binary
       index formula of Sec. 4), TT-SVD, rounding, sums, inner products.
qtt    an independent QTT construction of the stiffness operator A and load b
       (Sec. 5.1-5.3, Alg. 1) by TT-SVD of 1D factor matrices.
amen   O2: a plain alternating minimal-energy (AMEn) sweep for A u = M f0
       (Alg. 2), every contraction written out with numpy.einsum.
rng    SplitMix64, the counter-based generator used for the random initial
       guess and residual-tensor draws of the sweep.

Parity status of each function is stated in its docstring; functions pinned by
the tests in ``tests/test_oracle_*.py`` say so.
"""
