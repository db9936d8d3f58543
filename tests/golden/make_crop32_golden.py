"""Write tests/golden/crop32_oracle.npz: the CPU oracle's exact objective,
source weights and gradient for the 32^3 crop of the 128^3 differentiation
workload (48 systems: 16 sources x 5, 7, 9 Hz, lambda = 0.12, ESTIMATE mode).

Calls only the oracle and the seeded input generator.  Run from the
repository root:  python tests/golden/make_crop32_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import wri_synth  # noqa: E402


def main():
    t0 = time.time()
    prob = wri_synth.make_config("crop32", seed=0)
    out = oracle.objective_grad(prob, mode="estimate", return_fields=False)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "crop32_oracle.npz")
    np.savez_compressed(path, J=out["J"], J_sys=out["J_sys"], alpha=out["alpha"],
                        g=out["g"][0].astype(np.float64),
                        note="oracle.objective_grad(make_config('crop32', seed=0), mode='estimate')")
    print(f"wrote {path} in {time.time() - t0:.1f} s, J={out['J']:.6e}")


if __name__ == "__main__":
    main()
