"""Writes adjoint_config4.npz: the FP64 reference adjoint (oracle/ only: the
C oracle for the patch history, the torch float64 model with autograd for
the gradients) of the adjoint workload -- the 512 x 256 refined case, 2000
base steps, objective = dx^2 * sum of n(t_final) over the wavelength-square
window at the seed, gradients w.r.t. the base seed, E0, A and beta.

    python tests/golden/make_adjoint_config4.py     (about 10 minutes)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from adjoint_cases import history, reference_gradients  # noqa: E402
from paper_2105_13276_amd import workloads as W  # noqa: E402


def main():
    cfg = W.config4(steps=2000)
    sb, _ = W.seeds(cfg, fine=False)
    w = W.window_weights(cfg)
    _, ext0, growth = history(cfg, sb)
    ref = reference_gradients(cfg, sb, w, ext0, growth, seg=45)
    g = np.array([[k, *v] for k, v in sorted(growth.items())], np.int64).reshape(-1, 5)
    np.savez_compressed(os.path.join(HERE, "adjoint_config4.npz"), F=ref["F"], E0=ref["E0"],
                        A=ref["A"], beta=ref["beta"], seed=ref["seed"].astype(np.float32),
                        ext0=np.array(ext0, np.int64), growth=g, steps=cfg["steps"])
    print("F %.9e  dF/dE0 %.6e  dF/dA %.6e  dF/dbeta %.6e  |dF/dseed| %.6e"
          % (ref["F"], ref["E0"], ref["A"], ref["beta"], np.linalg.norm(ref["seed"])))


if __name__ == "__main__":
    main()
