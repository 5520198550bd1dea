"""FP64 CPU oracle for the Seele hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct NumPy (float64) implementation of what the
hot path computes: per-view preprocessing (Sec. 3.1 "Preprocessing", the
EWA projection behind Eq. 2, SH colour, and the opacity-aware extent of
Eqs. 3-5 in Sec. 3.3), the per-tile depth order (Sec. 3.1 "Sorting"),
front-to-back blending (Eqs. 1-2), contribution-aware blending
(Sec. 3.4, Algorithm 1), the active-set selection of hybrid preprocessing
(Sec. 3.3 "Algorithm") and the adjoint used for fine-tuning (Sec. 3.5).

Only ``tests/``, the smoke entry point and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the HIP library and never
imports it; the only common dependency is the seeded input generator in
``synthetic/``.

Every function is pinned by tests against closed forms, library routines
(SciPy spherical harmonics, SciPy rotations, ``np.lexsort``/``sorted``),
brute force on tiny inputs, hand counts and central finite differences.
"Parity unpinned": the contribution-aware image's distance from the plain
image, which the paper bounds only in its (absent) appendix (the distance
is frozen from this oracle, not derived), and the values of FLIP's CSF and
feature-detector constants (``flip``), restated from a publication that is
not available here.
"""
from . import sh, project, binning, blend, adjoint, hp  # noqa: F401
from .project import project_view, DEFAULTS  # noqa: F401
from .binning import bin_and_sort  # noqa: F401
from .blend import render_tiles, render_view, brute_force_view  # noqa: F401
