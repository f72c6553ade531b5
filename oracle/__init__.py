"""Plain, slow FP64 CPU oracle for shifted solves with a reused SPAI preconditioner.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``libmorx``) and imports nothing from it.

What it computes, following Singh & Ahuja, "Reusing Preconditioners in
Projection based Model Order Reduction Algorithms":

* ``pattern``    -- the static sparsity pattern shared by every factor
                    (pattern(A) plus the diagonal).
* ``spai``       -- SPAI as n independent column least-squares problems
                    (Section III-A, eqs. gen-precond / gen-precond-par) and the
                    reuse update ``min ||A_{i-1} - A_i Q_i||_F`` solved column by
                    column (Section III-B, Table 2 second approach; Section
                    III-C horizontal and vertical directions).
* ``precision``  -- rounding of factor values to FP32 / BF16 storage.
* ``chain``      -- the order in which factors make up the preconditioner of
                    shift i in round z (Algorithm 4) and its application as a
                    sequence of sparse products, never formed (Section III-B).
* ``bicg``       -- right-preconditioned two-sided BiCG for (sigma E - A) x = b
                    and its transpose (Section III-A, right preconditioning).
* ``projection`` -- two-sided Petrov-Galerkin projection and transfer functions
                    (Section II, interpolation of H and H').
* ``job``        -- a whole multi-round shifted-solve job in the paper's order.
* ``second_order`` -- AIRGA's solves (Algorithm 1, lines 4 and 10) for a
                    proportionally damped second-order model, with the same
                    reuse on its matrices ``s^2 M + s D + K``.

Every floating-point step is IEEE FP64 unless a storage precision is asked for.
Parity status of each function is stated in its module docstring.
"""
