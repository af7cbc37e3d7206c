"""FP64 CPU oracle for w-projection imaging -- TEST INFRASTRUCTURE ONLY.

This package is the independent correctness reference for the GPU library.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import it; the product path (the C-ABI library and its Python binding) never
does, and the two share no code.  Everything is float64.

Contents:
  pswf        zeroth-order prolate spheroidal wave function (the taper)
  wproj_ref   the imaging steps written out plainly: w-planes, kernel tables,
              per-visibility snapping, gridding, centred inverse DFT, grid
              correction, model-image-to-grid, degridding, chi^2 gradient
  eq56        the paper's baseline index (Eq. 5) and start-index prefix sum
              (Eq. 6) with the regrouping they drive
  cref        ctypes loader for the plain C gridder/degridder (oracle/c/wref.c),
              used for full-size parity and as the timed CPU baseline

The paper (Lao et al. 2019) cites w-projection (Cornwell, Golap & Bhatnagar
2008) without writing out its mathematics; the formulation here is the
standard one, with every free choice stated in the docstrings.
"""
