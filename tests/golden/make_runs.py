"""Write the oracle's whole-run results that the GPU tests compare against
(tests/golden/runs.json).  Calls only the FP64 oracle (oracle/).

Runs (seeded Gaussian initial conditions, 2LPT at z = 19, all modified gravity screened):

* the FP64-checkable sub-runs of the two large workloads, at their particle spacing
  (2 Mpc/h) and cell size (1 Mpc/h): nDGP r_c H0 = 1 with 64^3 particles on a 128^3 mesh
  in L = 128 Mpc/h, 30 steps; f(R) |f_R0| = 1e-5 with scale-dependent growth, 64^3 / 128^3
  / 128 Mpc/h and 128^3 / 256^3 / 256 Mpc/h, 20 steps; LCDM at the same sizes and step
  counts for the boosts;
* the step-count study (Sec. 7.3): f(R) F5 and nDGP r_c H0 = 1 with 32^3 particles on a
  64^3 mesh in L = 200 Mpc/h, n = 10, 20, 30 steps, and LCDM at each n.

Stored per run: P(k) of the final particles (k, P, modes per bin, up to half the mesh
Nyquist frequency) and the final displacements u (Mpc/h) of 1024 seeded particle
indices; per modified-gravity run the boost P_MG / P_LCDM of the same size and n.

Usage: python tests/golden/make_runs.py [threads]   (a few minutes on 8 cores)
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import fftlib  # noqa: E402
from oracle.cola import Run  # noqa: E402
from oracle.pk import power_spectrum  # noqa: E402

SAMPLES = 1024


def runs():
    out = {}
    sub = dict(z_init=19.0, seed=1, screening=1)
    for n_p in (64, 128):
        base = dict(np1d=n_p, nmesh1d=2 * n_p, box=2.0 * n_p, **sub)
        if n_p == 64:
            out["ndgp_64_128_n30"] = dict(model=oracle.MODEL_NDGP, rc_h0=1.0, n_steps=30, **base)
            out["lcdm_64_128_n30"] = dict(model=oracle.MODEL_LCDM, n_steps=30, **base)
        out[f"fr5_{n_p}_{2 * n_p}_n20"] = dict(model=oracle.MODEL_FR, fr0_abs=1e-5, n_steps=20, **base)
        out[f"lcdm_{n_p}_{2 * n_p}_n20"] = dict(model=oracle.MODEL_LCDM, n_steps=20, **base)
    small = dict(np1d=32, nmesh1d=64, box=200.0, **sub)
    for n in (10, 20, 30):
        out[f"fr5_32_64_n{n}"] = dict(model=oracle.MODEL_FR, fr0_abs=1e-5, n_steps=n, **small)
        out[f"ndgp_32_64_n{n}"] = dict(model=oracle.MODEL_NDGP, rc_h0=1.0, n_steps=n, **small)
        out[f"lcdm_32_64_n{n}"] = dict(model=oracle.MODEL_LCDM, n_steps=n, **small)
    return out


def lcdm_partner(name):
    return "lcdm_" + name.split("_", 1)[1]


def main():
    fftlib.set_workers(int(sys.argv[1]) if len(sys.argv) > 1 else 1)
    res = {}
    for name, kw in runs().items():
        p = oracle.Params(**kw)
        r = Run(p).run()
        k, P, nm = power_spectrum(r.u, p)
        nb = p.nmesh1d // 4 + 1   # bins up to half the mesh Nyquist frequency
        idx = np.random.default_rng(p.np1d).choice(p.n_part, SAMPLES, replace=False)
        res[name] = dict(params=kw, k=k[:nb].tolist(), P=P[:nb].tolist(),
                         nmodes=nm[:nb].astype(np.int64).tolist(), sample=idx.tolist(),
                         u=r.u[:, idx].tolist())
        print(name, flush=True)
    for name, d in res.items():
        if not name.startswith("lcdm_"):
            d["boost"] = (np.array(d["P"]) / np.array(res[lcdm_partner(name)]["P"])).tolist()
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "runs.json"), "w") as f:
        json.dump({"generator": "tests/golden/make_runs.py (oracle/, FP64)", "runs": res}, f)


if __name__ == "__main__":
    main()
