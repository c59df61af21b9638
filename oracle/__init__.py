"""FP64 CPU oracle for dense Sim(3) alignment, its cost adjoint and the Sim(3)
pose-graph solve, and point correction (EC3R-SLAM mapping back end:
Sec. III-C.2 eq. (sim3), Sec. III-C.3 and Sec. III-E).

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the HIP path is checked against. Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. The product library never imports, links or calls anything here,
and nothing here imports the product library.

Modules
-------
sim3     : group operations through the 4x4 generator and ``scipy.linalg.expm``
umeyama  : weighted Umeyama closed form (Sec. III-C.2, eq. (sim3))
irls     : confidence mask/weights + Umeyama start + Huber IRLS Gauss-Newton
cost     : Huber-weighted alignment cost, its analytic gradient, and central
           finite differences
implicit : derivative of the solved pose with respect to the points and
           confidences (implicit function theorem, exact Huber Hessian)
pgo      : dense Gauss-Newton Sim(3) pose-graph solve (Sec. III-E)
depth    : points of a depth-map pair (unprojection with each submap's camera,
           Sec. III-C.1)
points   : point correction: submap points to the world frame, sparse-map
           replacement (Sec. III-C.3)
metrics  : pose-error measures used to compare two Sim(3) estimates
"""
