"""Plain FP64 CPU oracle for the discrete-dipole-approximation solve.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls, links or
executes anything in this package: only the tests, the smoke check of
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may use it.  It
shares no code with the HIP library (``paper_1202_3424_amd``); the only module
both sides read is ``workloads`` (seeded geometry and random draws, no DDA
arithmetic).

Contents (each function cites the passage of the DDSCAT 7.2 User Guide,
Draine & Flatau, arXiv:1202.3424, that it follows, and, where the guide only
names a result, the published source it names):

* ``dense``   -- lattice constants, LATTDR/GKDLDR polarizabilities, the
                 interaction tensor, dense assembly and LU solve, incident
                 field, Q_ext / Q_abs / Q_pha, closed-form Q_sca, the
                 normal-equation residual of the guide's stopping test.
* ``fftsolve`` -- the FFT embedding of the interaction matrix and the Krylov
                 solvers (BiCGSTAB, QMR for complex-symmetric A,
                 BiCGstab(2)), for targets too large for dense LU.
* ``mie``     -- Mie theory for a homogeneous sphere.
* ``adjoint`` -- gradients of Q_abs and Q_ext with respect to the per-site
                 permittivity, by the adjoint of the dense solve.
* ``farfield`` -- far-field amplitudes, the amplitude and Mueller matrices,
                 backscattering and averages over scattering directions.
* ``nearfield`` -- E_inc and the field of the dipoles on an extended lattice
                 volume, and the field along a line between lattice points.

Pins (``tests/test_oracle_*.py``, run with ``-m "not gpu"``) tie each function
to something other than itself: the guide's printed worked example, closed
forms, textbook limits, brute-force quadrature and finite differences.
"""
