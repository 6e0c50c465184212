"""CPU FP64 oracle for the H-matrix power-series EFIE solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of the method of Negi, Balakrishnan and Rao, "Fast
Power Series Solution of Large 3-D Electrodynamic Integral Equation for PEC
Scatterers" (arXiv:2109.04129), in complex128 NumPy/SciPy.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  It shares no code with the HIP library in ``paper_2109_04129_amd`` and
never imports it; the two meet only through the seeded inputs of
``workloads``.

Modules, each citing the passage it follows:

* ``constants``  -- free-space constants, e^{jwt} convention (Sec. II).
* ``rwg``        -- RWG basis functions on a triangle mesh (Sec. II, [19]).
* ``quadrature`` -- triangle quadrature rules (Radon 7-point, 3-point).
* ``potentials`` -- closed-form 1/R and rho/R integrals over a triangle
                    (singularity extraction for eqs. 2-3).
* ``efie``       -- Galerkin EFIE matrix entries (eqs. 2-3, 9).
* ``cluster``    -- octree clusters and the admissibility split (eq. 10).
* ``aca``        -- re-compressed ACA of admissible blocks (eqs. 11-12).
* ``hmatrix``    -- near/far split Z = Z_N + Z_F (eq. 13).
* ``scaling``    -- right scaling coefficients and Schur steps (eqs. 14-23).
* ``series``     -- power-series solve (eqs. 24-36) and the ratio test (eq. 45).
* ``planewave``  -- plane-wave excitation and monostatic RCS (Sec. V).
* ``mie``        -- Mie series for a PEC sphere (comparison of Sec. V.C.1).
"""
