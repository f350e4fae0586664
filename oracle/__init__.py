"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, deliberately unoptimised NumPy/SciPy implementation of what
the GPU path computes, used to check it.  Only ``tests/``, the smoke entry
point and the benchmark's CPU-baseline leg may import this package; the
product package never does, and this package imports nothing from it.  The
two share no code: the only common module is ``synth`` (seeded inputs).

Modules:
  fd      the discretised acoustic problem of the paper's FWI/LSRTM section
          (forward map, misfit, adjoint-state gradient, Born and its
          adjoint) and the closed forms it is pinned to.
  aa      Anderson acceleration (Algorithm 1 in both the alpha and gamma
          forms, Algorithm 2 with the lambda line search) and the
          multi-secant form.
  krylov  restarted GMRES, L-BFGS and dense BFGS (comparators).
  cnn     the learned preconditioner's 3x3 convolution network, written
          out with hand-derived backward.
"""
