"""Realisation ensemble of the C3 errors on C1 (run by hand on a GPU; not a
pytest module).

C1's wake (Re about 800) amplifies perturbations, so the error of a run
against the FP64 oracle after 500 steps depends on the particular rounding
realisation: any change to the FP32 arithmetic of a kernel gives another
realisation of the same distribution.  This script measures that
distribution: for each storage format it runs C1 from the library's initial
state (seed 0) and from K - 1 starts perturbed by eps_s N(0, 1) in every
population (FP32 1e-9, FP16 and BF16 1e-7: below the rounding noise that
the storage adds every step), and reports the errors against the oracle
after 100 steps (computed here) and after 500 steps (the stored run of
tests/golden/make_c1_500.py), as in tests/test_gpu_precision.py.

    python tests/precision_ensemble.py out.json [K]
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle as O  # noqa: E402
from paper_1904_02108_amd import workload as W  # noqa: E402

EPS = {0: 1e-9, 1: 1e-7, 2: 1e-7}


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def main(out_path, k_runs=8):
    import torch

    from paper_1904_02108_amd import lbmibm as L
    ref = np.load(os.path.join(HERE, "golden", "c1_500_steps.npz"))
    steps = int(ref["steps"])
    z, y, x = ref["cells"].T.astype(np.int64)
    wl = W.config("c1")
    p = O.params(wl.shape, wl.tau, bc=wl.bc, forcing=wl.forcing)
    pts = O.Points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter)
    f = O.init_equilibrium(p)
    O.run(p, f, pts, 0, 99)
    r100 = O.step(p, f, pts, 99)
    rho100, U100 = O.moments(p, f)
    res = []
    for storage in (0, 1, 2):
        for seed in range(k_runs):
            sim = L.Simulation(wl.shape, wl.tau, bc=wl.bc, storage=storage, forcing=wl.forcing,
                               max_points=wl.n_points, max_iter=max(wl.n_iter, 8))
            sim.set_points(wl.rest, wl.area, wl.body_off, wl.bodies, wl.n_iter)
            if seed:
                pops = sim.read("pops", pops_f64=True)["pops"]
                g = torch.Generator(device="cpu").manual_seed(1000 + seed)
                noise = torch.randn(pops.shape, generator=g, dtype=torch.float64)
                sim.write(pops=pops + EPS[storage] * noise.to(pops.device))
            sim.step(100)
            o = {k: v.cpu().numpy() for k, v in sim.read("rho", "vel", "force", "pt_du").items()}
            e100 = dict(vel=rel(o["vel"], U100), rho=rel(o["rho"] - 1, rho100 - 1),
                        du=rel(o["pt_du"], r100["du"]), force=rel(o["force"], r100["G"]))
            sim.step(steps - 100)
            o = {k: v.cpu().numpy() for k, v in sim.read("rho", "vel", "force", "pt_du").items()}
            e = dict(storage=storage, seed=seed, at100=e100,
                     vel=rel(o["vel"][:, z, y, x], ref["vel"]),
                     rho=rel(o["rho"][z, y, x] - 1, ref["rho_minus_1"]),
                     force=rel(o["force"][:, z, y, x], ref["force"]),
                     du=rel(o["pt_du"], ref["du"]))
            sim.close()
            print(json.dumps(e), flush=True)
            res.append(e)
    with open(out_path, "w") as fh:
        json.dump(res, fh)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 8)
