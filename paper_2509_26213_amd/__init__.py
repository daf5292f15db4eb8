"""MI355X (gfx950) random-walker solver: C-ABI library librw.so + binding.

The hot path (matrix-free Jacobi-PCG of the random-walker Dirichlet problem,
batched brick solves, adjoint gradients) runs in the HIP kernels of
csrc/; this package only builds the library and marshals arguments.
"""
__all__ = ["rw", "build"]
