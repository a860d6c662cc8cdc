"""Plain FP64 CPU oracle of the multi-body double-layer Nystrom solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library; both sides only read the seeded descriptors produced by
``paper_2606_31380_amd.scenarios`` (inputs, no arithmetic of the method).

Modules (each function cites the passage of the paper it follows):

``geometry``   quasi-axisymmetric surface, Gauss-Legendre x trapezoid nodes,
               Jacobian, outward normals, rigid motions (Sections 2, 3.1, 6.2)
``modal``      modal Green's function and its source derivatives: toroidal
               Legendre functions by recurrence, elliptic integrals by AGM,
               FFT + convolution for k != 0 (Section 3.3)
``selfblock``  product-integration self-interaction block (Sections 3.1-3.4)
``pairsum``    inter-body double-layer pair sum (Section 4, display after
               the equation for the second part of the multi-body potential)
``solve``      plane-wave right-hand side, dense LU, right-preconditioned
               GMRES with the block-diagonal preconditioner, far field
               (Sections 4 and 6)

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against
closed forms (sphere double-layer eigenvalues, Mie series, Gauss's identity),
independent quadrature (mpmath) or brute force; none is "parity unpinned".
"""
