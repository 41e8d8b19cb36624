"""CPU oracle for the space-time reduced-order model (test infrastructure).

Plain, slow, FP64 NumPy/SciPy code that computes what the method computes,
step by step in the paper's order and notation (Choi, Brown, Arrighi,
Anderson, "Space-time reduced order model for large-scale linear dynamical
systems with application to Boltzmann transport problems").  It exists only
to check the HIP path: the tests, the package's smoke check and the CPU
baseline leg of the benchmark may call it; the product path never does.  It
shares no code with the HIP path and imports nothing from the package; both
sides receive the same seeded arrays as plain inputs.

Modules
-------
fom      full-order backward Euler (Sec. 2, Eq. (fom)) and the explicit
         space-time system (Eq. (st-fom), (stsystemmat), (ststate)).
pod      snapshot matrix, thin-SVD POD, temporal snapshot matrices and
         temporal bases (Sec. 4.1, Eq. (snapshotmat), (SVD), (temporalSVD)),
         with the completion rule for temporal bases wider than the data.
rom      spatial Galerkin operators (Sec. 3.1, Eq. (galerkin)), the explicit
         Kronecker space-time basis (Eq. (spacetimebasisvec)), brute-force
         projection (Eq. (st-galerkin)), the block formulas of Sec. 4.3,
         the reduced solve and the spatial-ROM time march.
bounds   the a-posteriori error bounds of Sec. 5 (Theorems 1-3).
cn       the Crank-Nicolson variant (the paper's remark that other time
         integrators give other block structures): full-order march,
         explicit space-time system and the reduced block formulas.
isvd     incremental SVD of a snapshot stream (Sec. 4.2, Alg. 1-2) and the
         spatial and temporal bases taken from it.
mlp      FP64 reference of the surrogate network (forward, hand-derived
         backward, Adam) used for gradient parity.

Every function names the passage it follows.  Readings where the paper is
silent or wrong are stated where they are used.
"""
