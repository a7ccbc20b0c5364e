"""Plain FP64 CPU oracle of range-separated stochastic-RI GF2 (RS-SRI-GF2).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check
and the CPU-baseline leg of the benchmark may import this package.  The
GPU library never calls into it, and it shares no code with the GPU path:
the only common module is ``chain_inputs`` (seeded synthetic inputs, none
of the method's arithmetic).

Every function states the part of the paper it follows (Dou, Chen,
Takeshita, Baer, Neuhauser, Rabani, "Range-Separated Stochastic Resolution
of Identity", arXiv 2005.12338).  Slow and obvious on purpose: no blocking
or fusion beyond what a definition states.

Modules
  rng         counter-based +-1 stochastic orbitals and uniforms
  integrals   RI factors K^Q (eq:K_ijQ, eq:vKQKQ) and the synthetic stand-in
  green       finite-temperature Green's function G(tau) (eq:Gij, eq:G0)
  split       range separation of K (eq:K_L) and of R (the L/S definitions)
  selfenergy  eq:sigma (brute force and bilinear form), eq:sigma_2 estimator
  energy      Galitskii-Migdal energy (eq:corr) and statistics
  proposal    importance proposal over the auxiliary index (project form)
  variants    control-variate and double-sum forms of the eq:sigma_2 average
  scf         Matsubara transforms, Dyson, mu tuning, RI Fock build (Section III)
  qp          quasiparticle energies: Pade continuation of the orbital self-energy
"""
