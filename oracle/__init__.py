"""CPU FP64 oracle for the FFCz dual-domain correction (test infrastructure only).

This package is the plain, slow reference that the HIP path is checked
against.  It is imported only by the test suite, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``; the product path never calls
it and shares no code with it.

Modules
-------
``ffcz``      the alternating projection of Alg. 1 (Sec. IV-B) step by step,
              the two projections, the bound verification, the FP32 closing
              clamp, the representability margin and the mask-based adjoint.
``dense``     the same loop written with explicit O(N^2) DFT matrices built
              from Eq. 1 / Eq. 3, used to pin ``ffcz`` on tiny grids.
``spectrum``  the shell-binned power spectrum of Sec. III and the
              log-spectrum loss used to exercise the adjoint.
``edits``     edit bookkeeping, CompactEdits, QuantizeEdits and the decoder
              (Alg. 1; Sec. IV-B, IV-D).
``bounds``    pointwise bounds, the disk variant and relative power-spectrum
              bounds (the footnote to Eq. 2; Sec. V-B).
``huffman``   the Huffman coding of the edit streams (LosslesslyCompressEdits).

Parity status: every function is pinned by a ``-m "not gpu"`` test
(brute-force DFT, Parseval, projection identities, regime closed forms,
a hand-worked N = 4 case, finite differences).  None is "parity unpinned".
"""

from . import ffcz, dense, spectrum  # noqa: F401
