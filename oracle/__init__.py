"""CPU float64 oracle for the RandRAND hot path — TEST INFRASTRUCTURE ONLY.

Plain, slow, readable numpy/scipy code that states what the GPU library
computes, step by step, in the paper's order and notation:

* rng        — counter-based generator for the random test matrices
               (SplitMix64 + Box-Muller, SRHT sign/sample descriptor).
* operators  — the operator A (stored dense, Gaussian RBF, Matern-3/2) and
               its shifted matvec A_mu u = A u + mu u.
* randrand   — sketch A_mu Omega, Cholesky QR and sketched (preconditioned)
               Cholesky QR, the C-RandRAND core G, refined projector T,
               the tau rules and the preconditioner apply; the joint basis
               for several shifts.
* solvers    — C-RandRAND PCG with restarts, plain CG, the direct Cholesky
               solve and residual certification.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library under
``paper_2509_19747_amd`` never imports it, and it never imports the library:
the two share no code.  The one common dependency is ``workloads`` (seeded
problem data with none of the method's arithmetic).
"""
