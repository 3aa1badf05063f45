"""FP64 CPU oracle for randomized HALS (Erichson, Mendible, Wihlborn, Kutz,
"Randomized Nonnegative Matrix Factorization", arXiv:1711.02037).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It exists so that the HIP library can be
checked against a plain, slow, obviously correct implementation written
directly from the paper.  Only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
The product path (``paper_1711_02037_amd``) never imports, calls or links it,
and this package never imports the product.  The two share no code.

Everything is NumPy in float64.  LAPACK (through ``numpy.linalg``) serves as
the textbook routine for the QR factorisation; every other step is the
algorithm of the paper written out in its own order and notation.

Readings of passages that are silent, ambiguous or misprinted are listed in the
module docstring of :mod:`oracle.rhals` and in the design document.

:mod:`oracle.adjoint` holds the reference gradients of unrolled sweeps: a
literal torch float64 transcription of the sweep differentiated by autograd
(readings R21-R23), pinned by central finite differences.

Parity status: every public function here is pinned by ``tests/test_oracle_pins.py``
against facts other than its own formula (closed forms, textbook routines,
brute-force minimisers, an independent library implementation of
coordinate-descent NMF, finite differences).  No function is "parity unpinned".
"""

from .rhals import (  # noqa: F401
    GRAM_FULL,
    GRAM_LOWDIM,
    GRAM_MIXED,
    ORDER_H_FIRST,
    ORDER_W_FIRST,
    NO_REG,
    Reg,
    clip,
    qr_positive,
    range_finder,
    compress,
    qb,
    qb_streaming,
    rhals_sweep,
    rhals_sweep_ordered,
    hals_sweep_ordered,
    order_blocked,
    order_interleaved,
    nndsvd,
    svd_init,
    hals_sweep,
    rhals,
    hals,
    projected_gradient_sq,
    projected_gradient_sq_compressed,
    rel_error,
    objective,
    sketch_width,
)
