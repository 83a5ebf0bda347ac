"""ORACLE -- test infrastructure only.

Plain, slow, obviously-correct CPU implementations of what the GPU library
computes, used to check it.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the product
path never does.  It shares no code with the GPU library.

Modules
-------
``sho``     the SHO kernel, its state-space matrices and the paper's
            closed-form discretisation (Appendix B), evaluated in mpmath.
``dense``   the dense integrated GP: the double integral of the kernel over
            each pair of exposure windows by Gauss-Legendre quadrature,
            Cholesky log-likelihood, posterior and analytic gradient.
``kalman``  ctypes wrapper around ``kalman.c``: the sequential augmented
            Kalman filter / RTS smoother / Algorithm-1 prediction in long
            double.
"""
