"""Plain FP64 CPU oracle for the lattice Dirac operators and solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or runs
this package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP library: its only dependency in
this repository is the seeded input generator module `synth`.

Every function follows the paper's definitions written out directly (numpy
`roll` over a (Lt, Lz, Ly, Lx, ...) array, `einsum` for colour and spin
algebra), in FP64, with no even-odd blocking, fusion or reordering beyond what
the definition states.  Sections cited are those of arXiv:2201.09004
("Performance of the GPU inverters with Chroma+QUDA for various fermion
actions"); standard lattice conventions the paper leaves unstated are marked
"(std)".

Modules:
  lattice    gamma matrices (chiral basis), shifts with boundary signs, parity
  wilson     Wilson D_W (eq. 2), clover term (eq. 3), twisted mass (eq. 1),
             even-odd Schur operator
  staggered  HISQ fat + Naik staggered operator (eq. 4, sec. 2.2), MILC and
             CPS phase conventions, even-site normal operator
  overlap    H_W = gamma5 D_W(-rho), Chebyshev approximation of the sign
             function (sec. 2.3, Fig. 2), massive overlap operator
  solve      plain CG / BiCGStab / multi-shift reference solvers, residuals
  dense      a deliberately naive per-site loop builder of dense matrices for
             brute-force checks on tiny lattices

Parity unpinned: the clover sign and its trace projection, and the HISQ
generator coefficients, are conventions that no printed number fixes; they are
pinned only internally (closed form of a constant field, hermiticity).
"""
