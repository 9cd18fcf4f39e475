"""CPU oracle for the reduced scattering system (RED / ORI).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference written from the paper (Ramm & Tran, "A Fast Algorithm for Solving
Scalar Wave Scattering Problem by Billions of Particles", arXiv:1602.04691).
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The GPU library never imports, links or calls
anything here, and nothing here imports the GPU library: the two share no code.

Everything is complex128 / float64 NumPy, with LAPACK (``numpy.linalg.solve``,
the singular values and the ``zgecon`` condition estimate) as the only library
primitive beyond ``numpy.fft`` in the Section 3 route.  ``rows.py`` spreads
independent sampled rows of eq. 2.19 over forked worker processes; each row's
arithmetic is the single-process function's.  ``fft_baseline.py`` is not
part of the definition: it runs the paper's own method (the convolution
product of Section 3, with ``scipy.fft`` on all host cores) as the
same-method CPU baseline of ``bench.py``, pinned against the dense sum.

Parity pins: every function is pinned by a CPU test in
``tests/test_oracle_pins.py`` or ``tests/test_physics_pins.py`` (no function
is "parity unpinned").
"""

from .ori_oracle import (  # noqa: F401
    C_S,
    cell_points,
    cell_volume,
    green,
    coupling,
    symmetric_scale,
    green_matrix,
    system_matrix,
    symmetric_system_matrix,
    solve_direct,
    condition_number,
    scatter_dense,
    sample_scatter_rows,
    sample_residual_rows,
    brute_force_system,
    gauss_solve,
    cocg,
    solve_symmetrized_cocg,
    objective,
    adjoint_gradient_dense,
)
from .section3 import (  # noqa: F401
    mirror_pad_axis,
    zero_pad_axis,
    green_table,
    convolve_section3,
    scatter_section3,
)
from .rows import sample_rows_parallel  # noqa: F401
from .fft_baseline import (  # noqa: F401
    green_spectrum,
    GreenConvolution,
    scatter_fft,
    solve_symmetrized_fft,
)
from .physics import (  # noqa: F401
    sqrt_branch_0_2pi,
    refraction_from_h,
    h_for_refraction,
    cell_charges,
    particle_charge,
    scattered_field,
    far_field,
    coarse_cell_of,
    interpolation_difference,
)
