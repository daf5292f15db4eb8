"""CPU oracle of the random-walker solve — TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import, call, link or run anything in this package.  The GPU library shares no
code with it and never calls it.

* rw_oracle.py      assembled-matrix NumPy/SciPy oracle (direct and step-by-step
                    Jacobi-PCG solves, hierarchy, adjoint gradient, complex step,
                    Monte-Carlo walks)
* rw_oracle_c.c     matrix-free float64 Jacobi-PCG with OpenMP (large grids, CPU timing)
* c_oracle.py       its ctypes front end
* exact_rational.py exact-arithmetic solve for the golden fixtures
"""
