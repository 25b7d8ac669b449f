"""CPU FP64 oracle for shift-invert spectrum slicing (arXiv:1908.06043).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

It is a plain, slow, obviously-correct restatement of what the method computes,
in the paper's order and notation, sharing no code with the HIP library:

* ``bk``       -- unblocked Bunch-Kaufman LDL^T of A - sigma B and the Sylvester
                  inertia read from D (Section 2.1 "major cost" factorization;
                  Section 2.2 inertia count);
* ``sisubit``  -- CholeskyQR, the shift-invert subspace iteration of Algorithm 2,
                  Rayleigh-Ritz and residuals (Section 2.1);
* ``validate`` -- candidate selection at tau and the three validation cases
                  (Section 2.2);
* ``kpm``      -- stochastic Chebyshev (KPM) density of states, the closed-form
                  CDOS, equal-count roots (eq. cdos_root) and interval midpoints
                  (Section 3.1 shift placement, with KPM standing in for the
                  Lanczos DOS);
* ``kmeans``   -- Lloyd's k-means and k-means++ seeding for shift migration
                  (Section 3.2);
* ``prng``     -- SplitMix64, the counter-based generator both sides implement;
* ``sislice``  -- the per-pencil driver: factor every shift, run Algorithm 2 per
                  probe until its window converges, validate, return the lowest n_e;
* ``dos``      -- the paper's own planner: Gaussian-broadened Lanczos DOS and its
                  closed-form CDOS (eq. dos, eq. cdos), equal-count roots, and
                  DOSCluster with refinement, safeguards and DOS-expectation
                  shifts (Section 3.1);
* ``scf``      -- probe migration between SCF steps (k-means clusters mapped to
                  probes by overlap, merge, delete, insert by 2-means; Section 3.2)
                  and the partial-trace monitor (Section 3.3);
* ``adjoint``  -- gradients of a loss of the lowest eigenpairs with respect to A
                  and B (first-order perturbation theory of the pencil of Section 1;
                  not a step of the paper): the sum-over-states definition and the
                  projected-solve form.

Parity pins for every function live in ``tests/test_oracle_*.py``.  The KPM
moments of a non-diagonal operator are a stochastic estimate: beyond the
zero-variance diagonal case and the invariants tested there, their value is
"parity unpinned" (they are compared to the HIP path, not to the paper).
"""
