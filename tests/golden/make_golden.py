"""Write the stored oracle results the GPU tests compare against (calls only oracle/ and synth).

    python tests/golden/make_golden.py [c2_pm128] [c1_pm32]
    python tests/golden/make_golden.py --codec c2_pm128

For each workload: Zel'dovich ICs from the oracle's Philox noise, the FP64 PM run to a = 1 on
uncompressed particles, and the auto power spectrum of the final CIC density (shells 1..N_m/2).
Output: tests/golden/<workload>_pk.json.

With --codec: the same run through the FP32 step reference of the compressed step (oracle.twin:
load-encode with the workload's code widths, integer CIC, FP64 Poisson solve rounded to FP32,
move, re-encode and counting sort), i.e. the spectrum the compression itself gives without any
GPU kernel. Output: tests/golden/<workload>_codec_pk.json.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
import numpy as np  # noqa: E402

from oracle import ic, pm, power, twin  # noqa: E402
from oracle.cosmology import Cosmology, step_factors  # noqa: E402


def run(name: str) -> dict:
    cfg = synth.WORKLOADS[name]
    cosmo = Cosmology(cfg["omega_m"], cfg["omega_l"], h=cfg["h"], sigma8=cfg["sigma8"], n_s=cfg["n_s"])
    nm, npart = cfg["nm_side"], cfg["np_side"]
    t0 = time.time()
    x, p, _ = ic.zeldovich(npart, nm, cfg["box"], cosmo, cfg["a_init"], cfg["seed"])
    k0, p0, n0 = power.power_spectrum(pm.density_contrast(pm.cic_deposit(x, nm), npart**3), cfg["box"])
    r = pm.PMRun(x, p, nm, cosmo, cfg["a_init"], cfg["a_final"], cfg["n_steps"], cfg.get("spacing", 0))
    while r.j < r.n_steps:
        r.advance()
        if r.j % 10 == 0:
            print(f"{name}: step {r.j}/{r.n_steps} {time.time() - t0:.0f}s", flush=True)
    delta = pm.density_contrast(pm.cic_deposit(r.x, nm), npart**3)
    k, pk, nmodes = power.power_spectrum(delta, cfg["box"])
    return dict(workload=name, config=cfg, a=cfg["a_final"], k=k.tolist(), pk=pk.tolist(), nmodes=nmodes.tolist(),
                k_init=k0.tolist(), pk_init=p0.tolist(), source="oracle: ic.zeldovich + pm.PMRun + power.power_spectrum",
                seconds=time.time() - t0)


def run_codec(name: str) -> dict:
    cfg = synth.WORKLOADS[name]
    cosmo = Cosmology(cfg["omega_m"], cfg["omega_l"], h=cfg["h"], sigma8=cfg["sigma8"], n_s=cfg["n_s"])
    nm, npart, nc = cfg["nm_side"], cfg["np_side"], cfg["nc_side"]
    nchi, nnu = cfg["x_bytes"], cfg["v_bytes"]
    t0 = time.time()
    x, p, _ = ic.zeldovich(npart, nm, cfg["box"], cosmo, cfg["a_init"], cfg["seed"])
    drift0, kicks, drifts = step_factors(cosmo, cfg["a_init"], cfg["a_final"], cfg["n_steps"], cfg["spacing"])
    st = twin.load(x, p, nc, nchi, nnu)
    st = twin.move(st, np.zeros((nm,) * 3, np.float32), np.float32(0.0), np.float32(drift0))
    for j in range(cfg["n_steps"]):
        delta = twin.delta_from_rho(twin.deposit_int(st, nm), st.n, nchi).astype(np.float64)
        phi = pm.poisson(delta, cfg["omega_m"]).astype(np.float32)
        st = twin.move(st, phi, np.float32(-kicks[j] / 12.0), np.float32(drifts[j]))
        if (j + 1) % 10 == 0:
            print(f"{name} codec: step {j + 1}/{cfg['n_steps']} {time.time() - t0:.0f}s", flush=True)
    delta = twin.delta_from_rho(twin.deposit_int(st, nm), st.n, nchi).astype(np.float64)
    k, pk, nmodes = power.power_spectrum(delta, cfg["box"])
    return dict(workload=name, config=cfg, a=cfg["a_final"], k=k.tolist(), pk=pk.tolist(), nmodes=nmodes.tolist(),
                source="oracle: ic.zeldovich + twin.load/move (FP32 step reference, the workload's codes) with "
                       "pm.poisson rounded to FP32 + power.power_spectrum",
                seconds=time.time() - t0)


if __name__ == "__main__":
    args = sys.argv[1:]
    codec = "--codec" in args
    names = [a for a in args if a != "--codec"] or ["c1_pm32", "c2_pm128"]
    for name in names:
        out = run_codec(name) if codec else run(name)
        fname = f"{name}_codec_pk.json" if codec else f"{name}_pk.json"
        with open(os.path.join(HERE, fname), "w") as f:
            json.dump(out, f, indent=1)
        print(f"wrote {fname} in {out['seconds']:.0f}s")
