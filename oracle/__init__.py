"""FP64 CPU oracle for one time step of differentiable cosmological hydrodynamics
(Horowitz & Lukic, "Differentiable Cosmological Hydrodynamics for Field-Level Inference and
High Dimensional Parameter Constraints", arXiv:2502.02294).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2502_02294_amd``: HIP kernels behind a C ABI) never imports it, and the two share
no code, headers, tables or constants.

The oracle is written in plain PyTorch CPU tensor operations in float64, one function per
step of the method in the paper's order, with no blocking, fusion or reordering.  Because
every step is an ordinary differentiable tensor expression, ``torch.autograd`` applied to
the oracle gives the exact reverse-mode derivative of the same discrete algorithm; that is
the oracle's adjoint (the paper differentiates its forward model the same way, by reverse
mode through the discrete scheme, Sec. 2.3.5).

Modules
  cosmology  background expansion, growth factor, BBKS spectrum, sigma_8 normalisation (Sec. 2.1)
  philox     Philox-4x32-10 counter-based generator (Salmon et al. 2011), written from its
             published definition; supplies the white noise and the Gumbel/logistic noise
  hydro      comoving Euler fluxes, relaxing TVD sweep with RK2, van Leer limiter, Strang
             order, CFL speed (Sec. 2.3, 2.3.1-2.3.3)
  gravity    CIC deposit/read-out, FFT Poisson solve, central-difference gradient, kick and
             drift (Sec. 2.2)
  subgrid    stochastic star formation with SN heating and its Gumbel-softmax relaxation
             (Sec. 2.4)
  ics        Gaussian random field, Zel'dovich displacements and gas initial state (Sec. 2.1)
  sim        configuration, state, the full time step, run-to-scale-factor and the loss
  riemann    exact Riemann solver for the Sod shock tube (test reference, Toro's method)

Where the paper leaves a passage open, the function that takes a reading of it says so in
its docstring; the functions cite the section or equation they follow.
"""

from . import cosmology, philox, hydro, gravity, subgrid, ics, sim, riemann  # noqa: F401
