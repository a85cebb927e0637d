"""Write the converged lid-driven cavity fields the GPU's converged GSIS
solutions are compared with (tests/test_gpu_configs.py).

Configuration: 64x64 quads on [0,1]^2 stored as an unstructured face list, lid
(y = 1) moving +0.1 x, every wall diffuse at T = 1; reduced 2D distributions
on a 32^2 stretched grid on [-6,6]^2; hard spheres (omega 0.5); uniform
M(1, 0, 1) start; every cell kinetic; Kn 0.1 and 1.

The references are the oracle's GSIS iteration (Sec. 3.1: 400 pseudo-time
steps of the synthetic equations per outer iteration, local steps at cfl 0.5)
from the same start, stopped by the same rule as the GPU run, eps < 1e-6
(Sec. 4 eq. convergence_critertion).  A closed cavity's steady state is fixed
only up to its total mass, which the iteration does not conserve exactly
(the diffuse walls take their density from the previous iterate), so the
reference follows the same algorithm rather than another iteration to the
same equations.  Only oracle/ and gsis_inputs/ are called.

    python tests/golden/make_cavity_reference.py [Kn ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gsis_inputs as gi  # noqa: E402
import oracle  # noqa: E402

TOL = 1e-6


def reference(Kn, max_iter=6000):
    m = gi.quad_cavity_2d(64, 64, 0.1)
    grid = gi.velocity_grid(2, 32, 6.0, "stretched")
    O = oracle.Oracle(m, grid, Kn)
    S = oracle.SteadySolver(O, mode="gsis", n_inner=400, cfl=0.5)
    S.set_state(gi.uniform_W(m["n_cells"]))
    t = time.time()
    eps = None
    for it in range(1, max_iter + 1):
        eps = S.step()
        if it % 100 == 0:
            print("Kn %g: %d iterations, eps %s, %.0f s" % (Kn, it, eps, time.time() - t), flush=True)
        if it >= 5 and eps.max() < TOL:
            break
    if eps.max() >= TOL:
        raise RuntimeError("not converged: eps %s after %d iterations" % (eps, it))
    path = os.path.join(HERE, "cavity_converged_kn%g.npz" % Kn)
    np.savez_compressed(path, W=S.W, eps=eps, iterations=it, Kn=Kn, tol=TOL)
    print("wrote", path, "after", it, "iterations", flush=True)


if __name__ == "__main__":
    for kn in (sys.argv[1:] or ["1", "0.1"]):
        reference(float(kn))
