"""Write the oracle's solutions of the benchmark configurations to
tests/golden/config_<case>.json.  Calls only the CPU oracle (oracle/) and the
seeded input generators; nothing here comes from the GPU library.

Cases (Sec. 6 cubic-inclusion benchmark and its batched, random-sphere
variant; readings R11-R13 for the reference medium and the interfaces):
  c2_<scheme>_<contrast>_<interface>   64^3, inclusion side 32, E contrast 10
      or 1e3, sharp or tanh interface (half-width 1 voxel), C0 = phase mean,
      six Mandel unit loads (one, eps_12, for the smooth contrast-1e3 AFB
      case, whose ~4700 iterations per load are too many for the oracle's
      speed), stopped at r <= 1e-6: iterations, residual, mean stress per
      load, C_eff (Mandel) when all six loads are present;
  c3_afb_1e3       128^3, side 64, contrast 1e3, eps_12 = 1e-3, to r <= 1e-10:
      iterations, residual history, mean stress, and the strain and stress on
      three lines through the cell (x, y, z, through the centre and through
      an interface);
  c4_<n>           a Poisson(20)-sphere cell (seed 2000 + n, sphere E
      log-uniform in [1, 1e3]), n = 48 and 96, six Mandel unit loads, a
      fixed number of iterations (tol 0): mean stress and residual history.

Usage: python tests/golden/make_config_goldens.py <case> [<case> ...]
       python tests/golden/make_config_goldens.py --list
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import solve3d  # noqa: E402
from paper_2009_03762_amd import inputs  # noqa: E402

UNITS = inputs.mandel_unit_strains()
MANDEL = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])


def c2_cell(contrast, interface):
    lam, mu = inputs.cubic_inclusion(64, 32, 1.0, contrast, interface=interface, eps=1.0)
    l0, m0 = inputs.reference_medium_mean(1.0, contrast)
    return lam, mu, l0, m0


def c4_cell(n):
    E = inputs.poisson_spheres(n, 2000 + n)
    lam, mu = inputs.lame_from_young(E, 0.3)
    lo, hi = inputs.lame_from_young(E.min(), 0.3), inputs.lame_from_young(E.max(), 0.3)
    return lam, mu, 0.5 * float(lo[0] + hi[0]), 0.5 * float(lo[1] + hi[1])


C4_ITERS = {48: 200, 96: 100}


def lines(field, n):
    """Three lines of a (6, n, n, n) field: along x through the centre, along y
    through the centre, along z through the inclusion's face region."""
    c, q = n // 2, n // 4
    return {"x_centre": field[:, c, c, :].tolist(), "y_centre": field[:, c, :, c].tolist(),
            "z_face": field[:, :, q, c].tolist()}


def case_c2(name):
    _, scheme, contrast, interface = name.split("_")
    chi = float(contrast)
    lam, mu, l0, m0 = c2_cell(chi, interface)
    loads = [5] if (chi > 100 and interface == "smooth") else list(range(6))
    rows = []
    for J in loads:
        r = solve3d.solve_gfp(lam, mu, UNITS[J], l0, m0, scheme=scheme.upper() if scheme == "fb" else "AFB",
                              tol=1e-6, maxit=20000)
        rows.append({"load": J, "iters": r.iters, "residual": r.residual, "status": r.status,
                     "sig_mean": list(map(float, r.sig_mean))})
        print(f"  {name} load {J}: {r.iters} iterations, r = {r.residual:.3e}", flush=True)
    out = {"case": name, "n": 64, "side": 32, "contrast": chi, "interface": interface, "scheme": scheme,
           "tol": 1e-6, "loads": rows}
    if len(loads) == 6:
        M = np.zeros((6, 6))
        for row in rows:
            M[:, row["load"]] = MANDEL * np.array(row["sig_mean"])
        out["ceff_mandel"] = M.tolist()
    return out


def case_c3(name):
    n = 128
    lam, mu = inputs.cubic_inclusion(n, n // 2, 1.0, 1e3)
    l0, m0 = inputs.reference_medium_mean(1.0, 1e3)
    Eb = inputs.macro_strain("12", 1e-3)
    r = solve3d.solve_gfp(lam, mu, Eb, l0, m0, scheme="AFB", tol=1e-10, maxit=5000)
    print(f"  {name}: {r.iters} iterations, r = {r.residual:.3e}", flush=True)
    return {"case": name, "n": n, "side": n // 2, "contrast": 1e3, "scheme": "afb", "tol": 1e-10,
            "ebar": list(map(float, Eb)), "iters": r.iters, "residual": r.residual, "status": r.status,
            "history": list(map(float, r.history)), "sig_mean": list(map(float, r.sig_mean)),
            "eps_lines": lines(r.eps, n), "sig_lines": lines(r.sig, n)}


def case_c4(name):
    n = int(name.split("_")[1])
    lam, mu, l0, m0 = c4_cell(n)
    K = C4_ITERS[n]
    rows = []
    for J in range(6):
        r = solve3d.solve_gfp(lam, mu, UNITS[J], l0, m0, scheme="AFB", tol=0.0, maxit=K)
        rows.append({"load": J, "history": list(map(float, r.history)), "sig_mean": list(map(float, r.sig_mean))})
        print(f"  {name} load {J}: r_K = {r.residual:.3e}", flush=True)
    M = np.zeros((6, 6))
    for row in rows:
        M[:, row["load"]] = MANDEL * np.array(row["sig_mean"])
    return {"case": name, "n": n, "seed": 2000 + n, "iters": K, "loads": rows, "ceff_mandel": M.tolist()}


CASES = ["c2_afb_10_sharp", "c2_fb_10_sharp", "c2_afb_10_smooth", "c2_fb_10_smooth", "c2_afb_1000_sharp",
         "c2_fb_1000_sharp", "c2_afb_1000_smooth", "c3_afb_1e3", "c4_48", "c4_96"]


def main(argv):
    if not argv or argv[0] == "--list":
        print("\n".join(CASES))
        return
    for name in argv:
        if name not in CASES:
            raise SystemExit(f"unknown case {name}")
        t0 = time.time()
        fn = case_c2 if name.startswith("c2") else case_c3 if name.startswith("c3") else case_c4
        out = fn(name)
        out["oracle_seconds"] = time.time() - t0
        with open(os.path.join(HERE, f"config_{name}.json"), "w") as f:
            json.dump(out, f)
        print(f"{name}: written ({out['oracle_seconds']:.0f} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
