"""FP64 CPU oracle for MFA direct volume rendering (MFA-DVR).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code,
table or constant generator with the HIP library under
``paper_2204_11762_amd/``, and neither side imports the other.

What it computes (plain definitions, FP64 throughout):

* ``bspline``  -- knot-span search, the Cox--de Boor basis and its first
  derivative, and the value and analytic gradient of a tensor-product
  B-spline volume (the MFA model of Sect. 2.3; the value and gradient
  queries of Sect. 3.1 / Algorithm 1).
* ``raycast``  -- the fixed-point ray-cast model of Sect. 3.1: one ray per
  pixel, constant sample distance between the first and last sample inside
  the volume, normalisation to the unit cube, transfer-function lookup,
  Phong shading from the analytic gradient, front-to-back compositing and
  early ray termination (Algorithm 1).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, brute force, invariants or independent library
routines; none is "parity unpinned".
"""

from . import bspline, quant, raycast  # noqa: F401
