"""CPU FP64 oracle for the OEFE ChFSI hot path (test infrastructure only).

This package is a plain, slow, direct transcription of the mathematics of the
orthogonalized-enriched finite-element Kohn-Sham operator and the
Chebyshev-filtered subspace iteration, written with numpy/scipy in float64
(complex128 at a Bloch wavevector).  It exists only to check the HIP library:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP path and imports
nothing from it.

Modules
-------
quadrature   GLL / Gauss rules and 1D Lagrange bases (Sec. III.A, eqnorthCGLL).
mesh         structured periodic hex mesh, DoF map, lumped GLL mass (eqnMcc).
potential    erf-smoothed nuclear potential at quadrature points.
enrichment   cutoff, atomic enrichment, orthogonalization, M^oo / H^co / H^oo
             (eqnUOEFEAtomic, eqnKSAtomicTrunc, eqnorthC, eqnorthCGLL, eqnMoo,
             eqnHOEFEelelements).
operator     the symmetrized operator M^-1/2 H M^-1/2 (eqnKSEigGenDiscrete,
             eqnKSEignStandDiscrete, eqnMOEFEInv), by cells and as CSR.
chfsi        Lanczos bounds, scaled Chebyshev filter, Cholesky-Gram-Schmidt,
             Rayleigh-Ritz and the pass driver (Sec. IV, eqnProjKS).
adjoint      band energy and its gradients w.r.t. V and X (eqnrho, E_band).
occupations  Fermi-Dirac occupations, Fermi level from the electron count, band
             energy and density from Ritz pairs (eqnfd, eqnne, eqnrho, E_band).
uform        the k-point Hamiltonian in the periodic-function form (eqnksdftu,
             eqnUOEFEAtomic, eqnHOEFEelelements with its k terms).
poisson      smeared nuclear charges and the auxiliary electrostatic potential in
             the OEFE basis (eqnsmeared, eqngr, eqnvg, eqnpoissonaux, eqnPhiOEFE,
             eqnpoissX, eqnDiscLaplace, eqnDiscForceVec).
adaptive     adaptive quadrature for the integrals of the enrichment functions
             (Sec. III.B) and the Kohn-Sham operator whose enrichment blocks use it.

Functions whose only check is agreement with the HIP path say "parity
unpinned" in their docstring.
"""
