"""FP64 CPU oracle of the fifth-order WENO finite-difference constrained-transport
MHD step (Donnert et al., "WENO-Wombat", arXiv:1812.04278).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code
with the HIP library and imports nothing from the product package.

Everything is float64 ``torch`` CPU tensors, vectorised over zones/faces; the
algorithm follows the paper's order and notation (Sect. 2, Appendix A), with
the readings of its garbled or silent passages listed in the header of
:mod:`oracle.mhd`.  Because it
is plain torch, ``torch.autograd`` through :func:`mhd.step` gives the reference
gradient used to check the hand-written adjoint.
"""
from . import mhd  # noqa: F401
