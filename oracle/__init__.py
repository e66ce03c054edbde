"""Independent FP64 CPU oracle for the boundary-integral Poisson-Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
never calls it and shares no code with it.

It computes, slowly and plainly, the dense collocation boundary-element
solution of the implicit-solvent model (Cooper & Barba, "Poisson-Boltzmann
model for protein-surface electrostatic interactions and grid-convergence
study using the PyGBe code"):

* ``units``      reduced units (lengths in A, charges in e, potentials in
                 e/(eps0 A)) and the SI conversions used at the boundary.
* ``quadrature`` triangle rules (1, 3, 4, 7 far points; 19 near points) and
                 Gauss-Legendre edge rules (Section 3.1, Discretization).
* ``integrals``  panel geometry, the near/far/self decision and the four
                 panel integrals V_L, K_L, V_Y, K_Y (eq. layers_element).
* ``bem``        dense block assembly of eq. matrix_phi / matrix_dphi for any
                 number of molecules and charged/potential surfaces, and of
                 Stern layers (one more interface per molecule), LU solve,
                 and the energies of Section 2 (eqs. solv_energy,
                 phi_reac_bem, energy_surf_disc, total_energy,
                 interaction_energy).
* ``analytic``   the two-sphere series solution of Section 4 and the
                 isolated-body closed forms (with a Stern shell too).
* ``adjoint``    gradients of the interaction free energy through the dense
                 transpose.

Pins (what fixes each part independently of itself) are in ``tests/``.
Every function here has such a pin; none is "parity unpinned".
"""
