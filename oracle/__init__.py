"""Plain FP64 CPU oracle for the relativistic lattice Boltzmann (RLBM) update.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The product library (``paper_1909_04502_amd``) never imports it and
shares no code, tables or constants with it.

Every routine here follows the paper (Gabbana, Simeoni, Succi, Tripiccione,
"Relativistic Lattice Boltzmann Methods: Theory and Applications",
arXiv:1909.04502) step by step, in the paper's order and notation, written for
readability rather than speed:

* ``mj``          Maxwell-Juettner integrals (App. B), equation of state
                  (Sec. 3, Eqs. defG / eos-ddim), Chapman-Enskog shear viscosity
                  (App. C).
* ``quadrature``  the quadrature rules (App. H printed ultra-relativistic rule;
                  product rules for the off-lattice scheme, a reading of
                  Sec. 5.3 where the paper is silent).
* ``basis``       Gram-Schmidt orthonormal polynomials and projection
                  coefficients (Sec. 5.2, Eqs. mj-feq-expansion,
                  mj-projection-coefficients, mj-discrete-feq).
* ``lattice``     the per-site time step of Sec. 6.2 (moments, Landau
                  eigenproblem, density, temperature, equilibrium, relaxation,
                  streaming) on a periodic / open grid, in torch float64 on CPU.
* ``grad``        reverse-mode gradient of a loss through the whole run
                  (autograd on the float64 CPU step; the eigenproblem and the
                  equation-of-state inversion are differentiated through one
                  Newton step at the converged solution).

Pins for every function live in ``tests/test_oracle_*.py`` (``-m "not gpu"``).
"""
