"""FP64 CPU reference implementation of the method (the oracle).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import, call or execute anything in this package; the
product library never does, and shares no code with it.

  modal.py      modal kernels k^S_m, k^D_m, k^G_m (Sec. 3.2)
  nystrom.py    single-body Fourier-mode Nystrom matrices and their inverses (Sec. 3.2)
  multibody.py  multibody block system, preconditioned operator, solves, fields (Secs. 3.3, 4)
  analytic.py   closed forms used to pin the above (Mie series, sphere eigenvalues)
  mlp.py        FP64 multilayer perceptron forward/backward (warm-start network)
  c/            FP64 OpenMP inter-body sum for large problems
"""
