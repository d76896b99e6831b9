"""spinmc oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct CPU reference for everything the HIP path of
``paper_2304_01772_amd`` computes.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
never does, and the two share no code (the seeded input generators live in
the separate ``synth`` package, which holds none of the method's arithmetic).

Contents
--------
* ``chain``       ctypes binding of ``spinmc_oracle.c`` (Philox, Metropolis
                  thresholds, Ising / Potts / Cellular Potts chains, integer
                  statistics).
* ``observables`` FP64 observables from integer statistics.
* ``gradients``   fluctuation (covariance) estimator of d<O>/d(theta).
* ``mlp``         FP64 reference of the 4-128-128-3 surrogate with the BF16
                  rounding points of the HIP kernels, its backward and Adam.
* ``dmc``         FP64 relaxed chain of the differentiable Monte Carlo
                  (Algorithm 2) with per-bond couplings, and its reverse-mode
                  gradients.
* ``spinopt``     FP64 energy with per-bond couplings, its gradient, the
                  quantised step, and the three spin-value optimisation
                  methods (annealed Monte Carlo, gradient, differentiable
                  Monte Carlo).

Parity status of every function is listed in its module docstring.
"""
