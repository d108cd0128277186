"""MI355X (gfx950) hot path of a randomized-preconditioned ensemble of
incremental 4D-Var assimilations: batched Lorenz-96 TL/AD Hessian products,
RHS-difference randomized Nystrom / REVD, spectral LMP and batched PCG, behind
the C ABI of include/eda.h.  The Python binding is in `eda`."""
