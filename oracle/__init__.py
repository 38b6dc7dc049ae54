"""CPU oracle of the modified D2Q9 lattice-Boltzmann scheme with the inlM stress.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports this; only
``tests/``, the smoke check and the CPU-baseline leg of the benchmark do.

* ``core``     ctypes binding of the FP64 C oracle (``lb_oracle.c``)
* ``analytic`` closed forms and quadratures from the paper (steady channel
               profile, simple shear, planar extension, Newtonian transients,
               cessation bound)
* ``mlp``      FP64 numpy forward/backward of the warm-start MLP
"""
