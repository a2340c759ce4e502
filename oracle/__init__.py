"""CPU oracle for the selected-SpMV path — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of everything the HIP
library computes, written from the paper (Elafrou, Goumas, Koziris, "A
lightweight optimization selection method for Sparse Matrix-Vector
Multiplication", arXiv 1511.02494).  It shares no code with the library under
``paper_1511_02494_amd/``: neither side imports the other.  Only the tests,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or execute anything in this package.

Modules
-------
``spmv``      plain sequential CSR SpMV (Algorithm 1) and a correctly rounded
              reference (error-free products + exact summation).
``features``  the structural features of Table 1, as exact integer
              accumulators and one fixed FP64 finalisation.
``select``    the profiling classifier's cascade (Section 3.2.1) and the
              class-to-optimisation map (Table 2).
``encode``    the derived formats: 16-bit column offsets (Section 3.3),
              merge-path split coordinates, x-block column slices and their
              long-row split, partitions, and FP32/BF16 value rounding.
``mlp``       the learned selector: input transform, FP32 forward pass with a
              fixed operation order, FP64 forward/backward and Adam.
``classic``   the paper's feature classifiers (Section 3.2.2): CART with the
              Gini criterion and Gaussian naive Bayes.
``cg``        conjugate gradients, the solver loop that amortises selection.
``cref``      ctypes wrapper of the plain C SpMV in ``csrc/spmv_ref.c``
              (the same loop, for host timing).

Parity status: every function is pinned by the tests under ``tests/``
(``-m "not gpu"``) except those whose header says "parity unpinned".
"""
