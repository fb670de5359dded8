"""libjfnk: Jacobian-free Newton-Krylov with a Jacobian-free geometric
multigrid preconditioner (Kothari, Kopanicakova, Krause, arXiv 2103.13890)
on one AMD MI355X.

The compute path is the C-ABI library ``libjfnk.so`` (HIP kernels for
gfx950, declared in include/libjfnk.h).  ``api`` is a thin ctypes binding
with the same entry-point names taking torch device tensors, and
``api.JFNKSolve`` wraps the solve and its adjoint as a
torch.autograd.Function; ``workloads`` generates the seeded synthetic
inputs.  Importing this
package does not load the library; the first call does, and it raises if
the library has not been built (there is no CPU fallback).
"""
__all__ = ['api', 'workloads', 'build']
