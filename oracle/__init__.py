"""Plain FP64 CPU oracle for the three pseudospectral schemes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The library's compute path never calls it, and the two share no
code: the oracle imports only numpy/scipy and the seeded input generators.

Each scheme is written out step by step in the order the paper states it
(Section "Fourier Pseudospectral Methods"), in float64/complex128, with a
library FFT (scipy's pocketfft) as the only primitive.  Where the paper is
silent or inconsistent, the reading taken is named in the docstring of the
function concerned.  Every function is pinned by a test in
``tests/test_oracle_*.py`` against values that the paper or the mathematics
fixes (worked example, closed forms, invariants, brute-force DFT).
"""

from . import spectral, nls, sg, ns  # noqa: F401
