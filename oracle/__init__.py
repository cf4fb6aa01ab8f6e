"""Plain FP64 CPU oracle for the f_obj(theta) hot path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything
under ``oracle/``.  The GPU library and its Python binding never import it,
and it imports nothing from them: the only code the two sides share is the
seeded input generator in ``workloads/``, which holds none of the method's
arithmetic.

Modules:
  model   -- Q_s, AR1, Kronecker, coregional mixing (Eq. 5, 6, 11), A, D,
             Q_p, Q_c (Eq. 1-4) in model order; BTA ordering
  linalg  -- dense and RCM+banded Cholesky (log-determinant, solve,
             selected diagonal of the inverse)
  fobj    -- f_obj(theta) of Eq. 8 and its parts
  laplace -- f_obj for a non-Gaussian (Poisson) likelihood: Newton search
             for the inner mode, Laplace approximation (Eq. 3, 4, 8)
  bfgs    -- central differences (Eq. 10) and BFGS on -f_obj (Eq. 9)
  mlp     -- FP64 reference of the surrogate network
"""
