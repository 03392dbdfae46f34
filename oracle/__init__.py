"""FP64 CPU oracle of the pseudo-potential lattice Boltzmann (P-LBM) update.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
definition of what the GPU path computes, written from the paper (Czelusniak,
Bingert, Krause, Simonis, "On the consistency of pseudo-potential lattice
Boltzmann methods", arXiv 2504.15018).  Only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` may import
it.  The product library never calls it and shares no code with it.

Everything is NumPy in float64, lattice units (dx = dt = c = 1, r = 1, G = -1),
whole-lattice array operations in the paper's step order:

  1. rho = sum_i f_i                                  eq. (Density)
  2. psi = sqrt(2 (rho/3 - p_EOS(rho)))              eq. (Interaction_Potential)
  3. M1, M2 over all directions of psi(x + c_i)       Sec. II, definitions of M^(1), M^(2)
  4. F = F^SC + eps/kappa corrections + F_g          eq. (interactionForce), reading R1
  5. u = (sum_i f_i c_i + F/2) / rho                  eq. (Momentum)
  6. tau(rho) linear in rho                           Sec. VI (relaxation-time interpolation)
  7. BGK (eq. LBE) or MRT collision with Guo forcing  eq. (Guo_Forcing_Scheme)
  8. streaming with periodic wrap or half-way bounce-back

Module map:
  lattice   velocity sets (eq. VelocitySet; D3Q19 extension)
  eos       paper EOS (eq. EOS), lattice Peng-Robinson EOS, psi
  params    unit converter (eqs. unit, unit2), K from width (eq. thickness),
            kappa from surface tension (eq. surface_tension), coexistence,
            generalised width / surface tension (derived from eq.
            New_Pressure_Tensor)
  step      the lattice update, moments read-out, initialisation
  mrt       moment bases for the MRT extension
  diag      global reductions (mass, momentum, max|u|, health flags)
  analytic  Appendix A profile, Appendix B surface tension, Young-Laplace,
            channel profile
  norms     error norms (eqs. relative_norms, norms)
  wellbalanced  the well-balanced discretisation (Sec. VI.B names the class
            of schemes; the reading is stated in the module): chemical-
            potential force and an equilibrium with a constant reference
            density on the moving populations

Readings of passages the paper leaves silent or prints garbled are listed in
the repository's design notes; the ones that change arithmetic are restated
where they are used.
"""
