"""CPU oracle for the nested Krylov-Ritz sign function (Bloch & Heybrock).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The library (``paper_0912_4457_amd``) never imports it and shares no
code with it; both read their inputs from ``nks_inputs``.

Plain, slow and written to be checked by eye against the paper: numpy/scipy
in float64/complex128, no blocking or fusion.  Modules:

* ``dirac``     -- gamma matrices and the explicit sparse A = gamma5 D_w(mu)
                   (Sec. 2, definition of D_w(mu)).
* ``signfun``   -- scalar sgn (Eq. sgnz), spectral matrix sign (Eq. fAdef),
                   Roberts-Higham iteration (Eq. Roberts).
* ``closedform`` -- free-field and pure-gauge sgn(A)b in momentum space
                   (derived from the definition of D_w(mu) and Eq. sgnz).
* ``krylov``    -- Lanczos (App. A) and two-sided Lanczos (App. B).
* ``precond``   -- p_opt, z'_max and improvement factors (Eqs. popt,
                   condimp, condimpNH; Sec. 4.1).
* ``nested``    -- the nested method of App. C (steps 2-6, no deflation),
                   the non-nested method (Eqs. non-nested, non-nested-oblique)
                   and the sgn^2 error estimate (Sec. 3).
* ``multilevel`` -- multi-level nesting k_0 -> k_1 -> ... -> k_L with p per
                   level (Sec. 4.5, Fig. 12).
* ``policy``    -- ell-doubling and k-checkpoint rules (not in the paper).
* ``mlp``       -- numpy MLP with bfloat16 weight rounding, forward, backward
                   and Adam (not in the paper).

Every function is pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_*``
against closed forms, printed numbers, library routines or invariants.
"""
