"""Writes gmres50_128cube.json: the oracle's restarted GMRES(50) on the DCGS2 basis for
the 3-D convection-diffusion workload (128^3 grid, v = (10, 10, 10), D = 1,
b ~ U(0,1) seed 3, x0 = 0, true relative residual 1e-8), in FP64 and with the basis
stored in FP32.  Only the oracle is called.

    python tests/golden/make_gmres_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import operators as ops  # noqa: E402
from oracle.gmres import gmres_dcgs2  # noqa: E402
from paper_2104_01253_amd import synth  # noqa: E402


def main():
    prob, b = synth.gmres_cd3d(128)
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    out = {"workload": "GMRES(50), 3-D convection-diffusion 128^3, v=(10,10,10), b~U(0,1) seed 3, "
                       "x0=0, rtol 1e-8 (true residual)", "restart": 50, "rtol": 1e-8}
    for name, qd in (("fp64", np.float64), ("fp32_basis", np.float32)):
        t0 = time.perf_counter()
        x, info = gmres_dcgs2(A, b, restart=50, rtol=1e-8, qdtype=qd)
        dt = time.perf_counter() - t0
        relres = float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
        out[name] = {"iters": int(info["iters"]), "cycles": int(info["cycles"]),
                     "relres_true": relres, "status": int(info["status"])}
        print(name, out[name], f"{dt:.1f} s", flush=True)
    with open(os.path.join(HERE, "gmres50_128cube.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
