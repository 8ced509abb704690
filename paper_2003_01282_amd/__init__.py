"""MI355X-native stochastic Lanczos quadrature (SLaQ, arXiv 2003.01282).

Submodules: `slaq` (binding of libslaq.so, the HIP library), `inputs`
(seeded synthetic graph workloads), `build` (compiles libslaq.so).  Importing
the package loads nothing; the library is loaded on first use.
"""
