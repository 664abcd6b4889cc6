"""Writes tests/golden/c5_adjoint_T64.json: the oracle's adjoint of the
full-size adjoint scene (262144 particles, 64^3 grid, 64 dithered substeps,
the c2 scheme) for the kinetic-energy objective and the centre of mass along
y (Sec. 6, Eqs. 8, 12-13).

Calls only the oracle and the input generators: the oracle runs its own
quantized trajectory (FP64 substeps, same codec and Philox draws), stores
every state s_0..s_64, and back-propagates through it.  Stored per objective:
z, per-field G = sum of lambda, g = sum of lambda^2 (Eq. 8), the per-field
ranges of the stored values (F - I for F), and lambda_0 of 512 particles
drawn with a fixed seed (columns in encode order).

    python tests/golden/make_c5_adjoint.py      # about 5 minutes on one core
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as orc  # noqa: E402
import workloads as WL  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_adjoint_T64.json")
T = 64
SAMPLE = 512


def trajectory(scene):
    sc, pr = scene["scheme"], scene["params"]
    w0, _ = orc.encode(sc, *scene["state"], 0, 2)
    sim = orc.Sim(sc, pr, w0)
    states = [orc.pack_state(*orc.decode(sc, w0))]
    for t in range(T):
        sim.step(1)
        st = orc.pack_state(*orc.decode(sc, sim.words()))
        out = np.empty_like(st)
        out[:, sim.ids()] = st
        states.append(out)
        if t % 8 == 7:
            print(f"forward step {t + 1}/{T}", flush=True)
    sim.close()
    return states


def main():
    scene = WL.c5(seed=0)
    states = trajectory(scene)
    rows = orc.field_rows(3)
    lo, hi = {}, {}
    for f, (a, b) in rows.items():
        vmin, vmax = np.inf, -np.inf
        for s in states:
            vals = s[a:b].copy()
            if f == "F":
                for k in range(3):
                    vals[4 * k] -= 1.0
            vmin, vmax = min(vmin, float(vals.min())), max(vmax, float(vals.max()))
        lo[f], hi[f] = vmin, vmax
    sample = np.sort(np.random.default_rng(2024).choice(scene["n"], SAMPLE, replace=False))
    out = {"scene": "workloads.c5(seed=0)", "steps": T, "sample": sample.tolist(), "lo": lo, "hi": hi,
           "objectives": {}}
    for kind, axis in (("ke", 1), ("com", 1)):
        z, G, g, A, lam0 = orc.adjoint_full(scene["params"], states, kind, axis)
        out["objectives"][kind] = {"axis": axis, "z": z, "G": G, "g": g,
                                   "lambda0_sample": lam0[:, sample].tolist()}
        print(f"{kind}: z={z:.9e} G={G} g={g}", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
