"""FP64 CPU oracle of the quasi-Newton / L-BFGS implicit-Euler step.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check of the package entry
file and the CPU-baseline leg of the benchmark may import anything from here.
The product path (the HIP library and its Python binding) never imports,
links or executes this package, and this package never imports the product.

The oracle is a plain, slow, NumPy/SciPy implementation written from the
paper (Liu, Bouaziz, Kavan, "Towards Real-time Simulation of Hyperelastic
Materials", 2016):

* materials.py -- Valanis-Landel energies and first Piola stresses
  (section 4.1, Eq. valanis-landel), signed SVD, and the stiffness rule
  (section 4.1, Eq. stiffness);
* fem.py       -- element precompute, lumped masses, the objective g and its
  gradient (section 3, Eq. PD; section 4, Eq. PDgrad2), and the constant
  matrix M/h^2 + L with its factorisation (section 3, Eqs. PDmatrixForm and
  PDsolution);
* solver.py    -- one time step: Algorithm 1 (quasi-Newton solver with
  backtracking Armijo line search) with Algorithm 2 (L-BFGS two-loop
  recursion) giving the descent direction (sections 4.1 and 4.2);
* newton.py    -- projected Newton iterated to convergence, used only to pin
  the minimiser on tiny meshes (section 5, Newton baseline and
  Eq. RelativeError).

Where the paper is silent or inconsistent, the readings used here are the
ones listed in the repository's design notes; each is named in a comment at
the place it applies.
"""
from .materials import (  # noqa: F401
    psi_and_P,
    signed_svd,
    stiffness,
    stress_profile,
)
from .fem import Model, build_model  # noqa: F401
from .solver import StepResult, step, two_loop, simulate  # noqa: F401
