"""Write the oracle's energy / enstrophy series of the 512 x 1024 workloads.

    OMP_NUM_THREADS=1 python tests/golden/make_series.py

Runs ONLY the FP64 oracle (``oracle/``) on the seeded inputs of
``cgp_inputs``: the one-layer workload (512 x 1024, levels 0, 1, 2, 1000
steps, dt 2.5e-5) and the two-layer workload (512 x 1024 per layer, levels
0, 1, 2, 500 steps).  Every ``every`` steps it records, per layer, the basin
energy of eq. 26 (of psi = P^l L_c^-1 R^l omega, the stream function the CGP
map gives the state) and the enstrophy, both divided by the basin area.  The
result, ``series_512x1024.json`` beside this script, is what the GPU horizon
tests compare the library's own diagnostics against.  The six runs are
independent and go to a process pool.
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

EVERY = 10
RUNS = [("c1", 0, 1000), ("c1", 1, 1000), ("c1", 2, 1000),
        ("c2", 0, 500), ("c2", 1, 500), ("c2", 2, 500)]


def run(job):
    import numpy as np

    import cgp_inputs as ci
    from oracle import diagnostics, model
    from oracle.grid import Grid
    from oracle.model import Physics

    name, level, nsteps = job
    case = ci.case_c1(level) if name == "c1" else ci.case_c2(level)
    g = Grid(case.nx, case.ny, case.lx, case.ly, case.y0)
    phys = Physics(inv_re=case.inv_re, inv_ro=case.inv_ro, f1=case.f1, f2=case.f2,
                   drag=case.drag)
    rng = np.random.default_rng(case.seed)
    w = ci.initial_field(case, rng)
    F = ci.forcing_field(case)
    two = case.nlayers == 2

    def stats(state):
        if two:
            psi = model.cgp_psi_two_layer(state, g, level, phys)
            return [[diagnostics.energy(psi[l], g), diagnostics.enstrophy(state[l], g)]
                    for l in range(2)]
        psi = model.cgp_psi(state, g, level)
        return [[diagnostics.energy(psi, g), diagnostics.enstrophy(state, g)]]

    t0 = time.time()
    steps, series = [0], [stats(w)]
    for n in range(1, nsteps + 1):
        w = (model.step_two_layer if two else model.step)(w, F, g, level, phys, case.dt)
        if n % EVERY == 0:
            steps.append(n)
            series.append(stats(w))
    return dict(workload=name, level=level, nsteps=nsteps, dt=case.dt, seed=case.seed,
                nlayers=case.nlayers, steps=steps, E_Z=series, seconds=time.time() - t0)


def main():
    with ProcessPoolExecutor(max_workers=len(RUNS)) as ex:
        out = list(ex.map(run, RUNS))
    doc = dict(
        source="FP64 oracle (oracle/model.py, oracle/diagnostics.py) on the seeded cgp_inputs "
               "workloads; written by tests/golden/make_series.py",
        quantity="per layer [E, Z]: eq. 26 kinetic energy of psi = P^l L_c^-1 R^l omega and "
                 "enstrophy 1/2 <omega^2>, both divided by the basin area",
        every=EVERY, runs=out)
    path = os.path.join(HERE, "series_512x1024.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", path, [round(r["seconds"]) for r in out])


if __name__ == "__main__":
    main()
