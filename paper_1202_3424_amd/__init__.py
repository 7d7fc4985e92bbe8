"""MI355X-native discrete-dipole-approximation solver.

The DDA scattering problem of the DDSCAT 7.2 User Guide (Draine & Flatau,
arXiv:1202.3424): N polarizable points on a cubic lattice, A P = E solved by
BiCGSTAB, QMR for complex-symmetric A or BiCGstab(2), whose matrix-vector
product is an FFT convolution with the lattice Green tensor plus the
lattice-dispersion-relation diagonal (LATTDR or GKDLDR); returns P and Q_ext,
Q_abs, Q_sca, Q_pha.  From P: far-field amplitudes and the Mueller matrix
(``far_field``, ``mueller``), Q_sca, g and <cos^2> over scattering directions
(``scattering_averages``), E in and around the target (``nearfield``,
``field_line``), and the gradient of Q_abs / Q_ext in the per-site
permittivity (``grad_eps``, ``QEff``).  Many targets and orientations go
through ``solve_batched``.  The compute path is libdda.so (HIP kernels for
gfx950 behind the C ABI of include/dda.h); this package only marshals
arguments.  ``paper_1202_3424_amd.build.build()`` compiles the library.

The public names below load libdda.so on first use and raise ImportError if
it has not been built: there is no fallback implementation.
"""
_PUBLIC = ("DDAError", "Options", "QEff", "Target", "apply", "apply_noalloc", "context", "far_field", "field_line", "get_timing",
           "grad_eps", "last_error", "mueller", "nearfield", "nearfield_volume",
           "scattering_averages", "set_timing", "set_timing_sample", "solve", "solve_batched", "solve_rhs",
           "tuned_variants")

__all__ = list(_PUBLIC)


def __getattr__(name):
    if name in _PUBLIC:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
