"""Write pd_inputs/params.json: the time step of every workload specimen and
the end-twist rate of the cylinder.  Calls only the CPU reference.

Time step rule (the stability bound delta/c' quoted with Eq. 2.13 is not
sufficient for this operator; the largest stable step of the explicit update
of Eq. 2.11 for an undamped linear system is 2/omega_max):

    lambda_max = power iteration on K x = lambda M x, free DOFs, intact
                 specimen (no notch), seed 0
    dt         = 0.8 * 2 / sqrt(1.001 * lambda_max), rounded down to four
                 significant digits

Cylinder twist rate: the end layers rotate by +-phi/2 with
phi(t_end) = 4 s_c L / r (surface principal strain 2 s_c), t_end = steps * dt.

usage: python -m oracle.make_params [key ...]     (default: every key)
"""

from __future__ import annotations

import json
import math
import sys
import time

import numpy as np

import pd_inputs
from pd_inputs import workloads as W

from .oracle import Oracle, critical_stretch


def floor4(x: float) -> float:
    e = math.floor(math.log10(x)) - 3
    return float("%.4g" % (math.floor(x / 10.0 ** e) * 10.0 ** e))


def stable_dt(w, iters: int = 500) -> float:
    o = Oracle(w, apply_cuts=False, dt=np.ones(w.n_specimens))
    lam = o.lambda_max(iters, 0)
    return floor4(0.8 * 2.0 / math.sqrt(1.001 * lam))


def compute(key: str, params: dict, iters: int):
    t0 = time.time()
    if key == "cantilever3d":
        params[key] = stable_dt(W.cantilever3d(dt=1.0), iters)
    elif key == "plate2d":
        params[key] = stable_dt(W.plate2d(dt=1.0), iters)
    elif key == "impact3d":
        params[key] = stable_dt(W.impact3d(dt=1.0), iters)
    elif key in ("cylinder3d", "cylinder3d_dx05"):
        dx = 0.6e-3 if key == "cylinder3d" else 0.5e-3
        w = W.cylinder3d(dx=dx, dt=1.0, twist_rate=0.0)
        dt = stable_dt(w, iters)
        mat = w.materials[0]
        s0 = critical_stretch(0, mat.E, mat.nu, mat.G0, w.delta, w.s0_variant)
        L, r = 100e-3, 25e-3
        phi_end = 4.0 * s0 * L / r
        params[key] = dt
        params[key + "_twist_rate"] = phi_end / (w.steps * dt)
    elif key == "batch2d":
        draws = W.batch_draws(256, 2309)
        out = []
        for k in range(len(draws)):
            w = W.batch2d(n_plates=1, first=k, dt=np.ones(1))
            out.append(stable_dt(w, iters))
        params[key + "_dt"] = out
    else:
        raise KeyError(key)
    print(f"{key}: done in {time.time() - t0:.1f} s", flush=True)


def main(argv):
    keys = argv or ["cantilever3d", "plate2d", "impact3d", "cylinder3d", "cylinder3d_dx05",
                    "batch2d"]
    iters = 500
    params = W.load_params()
    for k in keys:
        compute(k, params, iters)
        with open(W.PARAMS_PATH, "w") as f:
            json.dump(params, f, indent=1, sort_keys=True)
    print(json.dumps({k: v for k, v in params.items() if not isinstance(v, list)}, indent=1))


if __name__ == "__main__":
    main(sys.argv[1:])
