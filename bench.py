"""Throughput of the AFB fixed point on one MI355X.

Workload: 256^3 periodic cell, centred cubic inclusion of side 128 voxels
(sharp interface), inclusion/matrix Young's modulus 1e3 / 1, nu = 0.3 in both
phases, reference medium C0 = mean of the phase Lame moduli, macroscopic
shear eps_12 = 1e-3, PCD discretisation, AFB (= rotated) scheme.  One step is
one full fixed-point iteration; in the default displacement form: the stencil
kernel (strain from u, Hooke, divergence, forward x transform), forward y,
z-pass with the Green step, reduction of residual and mean stress, inverse y,
and the displacement update with the inverse x transform (`--form strain`:
x-pass with the strain update, Hooke and both x transforms, forward y, z-pass
with the Green step, reduction, inverse y).  The tolerance is 0, so exactly
`--steps` iterations run; inputs are resident in HBM before timing.

Prints one JSON line: value = GVoxel-iterations/s of the FP32 path (FP32
transforms and Green step, FP64 reductions); the FP64 path is reported under
"fp64".  "roofline" is for the dominant kernel, timed with HIP events on the
solver's stream inside the timed region.  "equal_accuracy" gives, for the
FP64 path and the FP32 paths (displacement form, the same with five FP64
warm-start iterations, strain form), the iterations and wall time needed to bring
the strain field within a relative L2 error of 1e-5 and 1e-6 of a tight FP64
solution, and the FP32 speedups at equal accuracy; its "certified_stop" rows
solve to r <= 1e-6 with the stopping test itself: FP64, and FP32 with FP64
iterations down to r = 3e-4 followed by FP64-refined F32 cycles of 8 (every
reported residual an FP64 evaluation).  "batched_ceff" times the effective
stiffness (six load cases) of 48 random cells of five sizes: plain FP64
solves (timed on a quarter of the cells, same size mix), all sizes in one
group graph in FP64 and in FP32, and FP32 with one stream per size group.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FIXED_BALG = 248.0  # bytes per voxel-iteration, FP32, of the six-component strain-form sweep


def workload(n):
    from paper_2009_03762_amd import inputs
    lam, mu = inputs.cubic_inclusion(n, n // 2, 1.0, 1e3, 0.3)
    l0, m0 = inputs.reference_medium_mean(1.0, 1e3, 0.3)
    Eb = inputs.macro_strain("12", 1e-3)
    return lam, mu, l0, m0, Eb


KERNEL_NAMES = {
    "strain": {0: "k_xpass", 1: "k_ypass(forward)", 2: "k_zpass", 3: "k_ypass(inverse)", 5: "k_reduce"},
    # the displacement form's reduction runs in the stencil's last workgroup
    "displacement": {0: "k_stencil", 1: "k_ypass(forward)", 2: "k_zpass_u", 3: "k_ypass(inverse)",
                     4: "k_uxpass"},
}


def algorithmic_bytes(kernel, n, esize, scheme="afb"):
    """Bytes a kernel must move per launch: one read and one write of every
    field it transforms or updates, one read of every field it only uses.
    Strain form: the x-pass reads and writes the six-component spectrum and
    the strain and reads the two moduli.  Displacement form: the stencil
    kernel reads u and the moduli and writes the three-component spectrum of
    div sigma; the update reads that spectrum and reads and writes u.  The
    displacement u is held in FP64 in both precisions."""
    n1 = n2 = n3 = n
    N = n1 * n2 * n3
    half = n3 * n2 * (n1 // 2 + 1) * 2 * esize  # one component of the half spectrum
    spec6, spec3 = 6 * half, 3 * half
    table = {
        "k_xpass": 2 * spec6 + 2 * 6 * N * esize + 2 * N * esize,
        "k_ypass(forward)": 2 * spec6,
        "k_ypass(inverse)": 2 * spec6,
        "k_zpass": 2 * spec6 + (21 * half // 2 if scheme == "dgo" else 0),
        "k_stencil": 3 * N * 8 + 2 * N * esize + spec3,
        "k_uxpass": spec3 + 2 * 3 * N * 8,
        "k_zpass_u": 2 * spec3,
        "k_ypass(forward)/3": 2 * spec3,
        "k_ypass(inverse)/3": 2 * spec3,
    }
    return table.get(kernel, 0)


def kernel_bytes(name, form, n, esize):
    if form == "displacement" and name.startswith("k_ypass"):
        return algorithmic_bytes(name + "/3", n, esize)
    return algorithmic_bytes(name, n, esize)


def bytes_per_iteration(n, esize, form="strain"):
    return sum(kernel_bytes(k, form, n, esize) for k in KERNEL_NAMES[form].values() if k != "k_reduce")


def source_sha():
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2009_03762_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, key, n, schedule):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    record (key: "f32" displacement form, "f32_strain" strain form), if it was
    taken on the current kernel sources, this workload and this launch
    schedule."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("source_sha") != source_sha() or n != 256:
        return None
    rs = rec.get("schedule", {}).get(key)
    if rs is None:
        return None
    # only the launch parameters of the kernel itself must match: the
    # stencil's planes per workgroup and its tile order (bit 0 of xcd_order)
    if kernel == "k_stencil":
        if (rs["stencil_planes"], rs["xcd_order"] & 1) != (schedule["stencil_planes"], schedule["xcd_order"] & 1):
            return None
    elif rs != schedule:
        return None
    ent = rec.get("kernels", {}).get(kernel, {}).get(key)
    if not ent:
        return None
    return ent["read_bytes"] + ent["write_bytes"]


def run_gpu(prec, n, steps, warmup, breakdown=True, form="displacement", autotune=True):
    import torch

    from paper_2009_03762_amd import lsfft
    lam, mu, l0, m0, Eb = workload(n)
    esize = 4 if prec == "f32" else 8
    torch.cuda.synchronize()
    s = lsfft.Solver(lam, mu, l0, m0, scheme="afb", disc="pcd", prec=prec, form=form)
    print(f"[bench] {prec}: solver created for {n}^3 ({form} form)", file=sys.stderr, flush=True)
    tuned = None
    if autotune:
        t0 = time.perf_counter()
        sched, ms0, ms1 = lsfft.autotune(s.handle, 16)
        tuned = {"schedule": sched, "default_ms_per_iter": ms0, "tuned_ms_per_iter": ms1,
                 "tune_seconds": time.perf_counter() - t0}
        print(f"[bench] {prec}: schedule {sched}: {ms0:.4f} -> {ms1:.4f} ms/iter", file=sys.stderr, flush=True)
    else:
        tuned = {"schedule": lsfft.get_schedule(s.handle)}
    s.solve_device(Eb, tol=0.0, maxit=warmup)
    torch.cuda.synchronize()
    names = KERNEL_NAMES[form]
    ids = {v: k for k, v in names.items()}
    kernels = {}
    if breakdown:
        for kid, name in names.items():
            lsfft.set_timing(s.handle, kid)
            s.solve_device(Eb, tol=0.0, maxit=10)
            ms, cnt = lsfft.get_timing(s.handle)
            kernels[name] = {"mean_ms": ms, "launches": cnt}
        dominant = max((k for k in kernels if k != "k_reduce"), key=lambda k: kernels[k]["mean_ms"])
    else:
        dominant = names[0]
    lsfft.set_timing(s.handle, ids[dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = s.solve_device(Eb, tol=0.0, maxit=steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_ms, dom_cnt = lsfft.get_timing(s.handle)
    lsfft.set_timing(s.handle, -1)
    T = t1 - t0
    N = n ** 3
    value = N * steps / T / 1e9
    ab = kernel_bytes(dominant, form, n, esize)
    achieved = ab / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else None
    res = {
        "value": value,
        "ms_per_step": T / steps * 1e3,
        "residual_final": out["residual"],
        "iters": out["iters"],
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": measured_traffic(dominant, prec if form == "displacement" else prec + "_strain", n,
                                        tuned["schedule"]),
            "bytes_per_launch": ab,
            "mean_launch_ms": dom_ms,
            "launches_timed": dom_cnt,
        },
        "whole_iteration_hbm_frac": value * 1e9 * bytes_per_iteration(n, esize, form) / N / (HBM_PEAK_GBS * 1e9),
        # the same with the fixed 248 B (FP32) / 496 B (FP64) per voxel-iteration of the six-component
        # strain-form sweep (strain read + write, moduli, four six-component spectrum sweeps)
        "whole_iteration_frac_fixed_balg": value * 1e9 * FIXED_BALG * (esize // 4) / (HBM_PEAK_GBS * 1e9),
        "bytes_per_voxel_iteration": bytes_per_iteration(n, esize, form) / N,
        "form": form,
        "kernels": kernels,
        "autotune": tuned,
    }
    s.close()
    torch.cuda.synchronize()
    return res


def equal_accuracy(n, targets=(1e-5, 1e-6), kmax=500, kstep=10):
    """Iterations and wall time each path needs to bring the strain field to a
    relative L2 error `target` against a tight FP64 solution (equilibrium
    residual 1e-10) of the same workload, every error measured on the GPU."""
    import torch

    from paper_2009_03762_amd import lsfft
    lam, mu, l0, m0, Eb = workload(n)
    shape = (6, n, n, n)
    ref = torch.zeros(shape, dtype=torch.float64, device="cuda")
    s = lsfft.Solver(lam, mu, l0, m0, scheme="afb", disc="pcd", prec="f64", form="displacement")
    r = s.solve_device(Eb, tol=1e-10, maxit=2000, eps_dev=ref)
    s.close()
    rn = torch.linalg.vector_norm(ref).item()
    out = {"reference": f"FP64 displacement form stopped at r = {r['residual']:.2e} after {r['iters']} iterations",
           "metric": "relative L2 error of the strain field", "paths": {}}
    print(f"[bench] accuracy reference: {out['reference']}", file=sys.stderr, flush=True)
    for name, prec, form, warm in (("f64", "f64", "displacement", 0), ("f32", "f32", "displacement", 0),
                                   ("f32_warm5", "f32", "displacement", 5), ("f32_strain", "f32", "strain", 0)):
        dt = torch.float64 if prec == "f64" else torch.float32
        e = torch.zeros(shape, dtype=dt, device="cuda")
        s = lsfft.Solver(lam, mu, l0, m0, scheme="afb", disc="pcd", prec=prec, form=form, f64_warmup=warm)
        s.solve_device(Eb, tol=0.0, maxit=5, eps_dev=e)
        found = {}
        curve = []
        k = kstep
        while k <= kmax and len(found) < len(targets):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.solve_device(Eb, tol=0.0, maxit=k, eps_dev=e)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            err = (torch.linalg.vector_norm(e.double() - ref) / rn).item()
            curve.append((k, err))
            for t in targets:
                if t not in found and err <= t:
                    found[t] = {"iters": k, "ms": ms, "field_err": err}
            k += kstep
        s.close()
        del e
        out["paths"][name] = {"form": form, "prec": prec, "f64_warmup_iters": warm,
                              "targets": {f"{t:g}": found.get(t) for t in targets},
                              "err_curve": [[k, float(f"{v:.3e}")] for k, v in curve]}
        print(f"[bench] accuracy {name}: {out['paths'][name]['targets']}", file=sys.stderr, flush=True)
    speed = {}
    for t in targets:
        key = f"{t:g}"
        base = out["paths"]["f64"]["targets"][key]
        for name in ("f32", "f32_warm5", "f32_strain"):
            got = out["paths"][name]["targets"][key]
            if base and got:
                speed[f"{name}@{key}"] = base["ms"] / got["ms"]
    out["speedup_over_f64"] = speed
    # solves stopped by the stopping test at r <= 1e-6 (reading R2): F64, and
    # F32 certified by FP64 evaluations (FP64 iterations until r <= 3e-4,
    # then refinement cycles of 8)
    tol = 1e-6
    rows = {}
    for name, kw in (("f64", dict(prec="f64")),
                     ("f32_until3e-4_refine8", dict(prec="f32", f64_until=3e-4, refine=8))):
        dt = torch.float64 if kw["prec"] == "f64" else torch.float32
        e = torch.zeros(shape, dtype=dt, device="cuda")
        s = lsfft.Solver(lam, mu, l0, m0, scheme="afb", disc="pcd", form="displacement", **kw)
        s.solve_device(Eb, tol=tol, maxit=1000, eps_dev=e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = s.solve_device(Eb, tol=tol, maxit=1000, eps_dev=e)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        err = (torch.linalg.vector_norm(e.double() - ref) / rn).item()
        s.close()
        del e
        rows[name] = {"status": lsfft.status_string(o["status"]), "iters": int(o["iters"]),
                      "residual": float(o["residual"]), "ms": ms, "field_err": err}
        print(f"[bench] certified stop {name}: {rows[name]}", file=sys.stderr, flush=True)
    rows["f32_speedup_over_f64"] = rows["f64"]["ms"] / rows["f32_until3e-4_refine8"]["ms"]
    out["certified_stop"] = {"tol": tol, "rows": rows}
    del ref
    torch.cuda.synchronize()
    return out


def batched_ceff(ncells=48, seed0=1000, tol=1e-6, plain_stride=4):
    """Effective stiffness (six unit load cases) of `ncells` random cells:
    sizes drawn from {32, 48, 64, 96, 128}^3, Poisson(20) spheres of radius
    U[3, 8] voxels, log10 E uniform in [0, 3] per sphere, matrix E = 1,
    nu = 0.3, C0 = mean of the Lame moduli of the extreme E, AFB.  Paths,
    solve time only (handles created beforehand):
      plain   FP64, one solve per load case and cell (tol), timed on every
              `plain_stride`-th cell (the same size mix): its rate in
              GVoxel-iter/s prices the whole set;
      group   one batch handle per cell size holding every cell and load case,
              all sizes solved by lsfft_solve_group (one graph launch per
              chunk of iterations over every size): FP64 to tol (the
              reference C_eff), and FP32 with five FP64 warm-start iterations
              run for the largest FP64 iteration count of each size group
              (the FP32 residual cannot certify tol at these contrasts);
      streams the same FP32 handles, each size group solved by its own host
              thread on its own stream (the previous way to overlap sizes);
    with each path's C_eff error against the FP64 group reference."""
    import torch
    from concurrent.futures import ThreadPoolExecutor

    from paper_2009_03762_amd import inputs, lsfft
    rng = np.random.default_rng(seed0)
    sizes = [32, 48, 64, 96, 128]
    cells = []
    for b in range(ncells):
        n = int(rng.choice(sizes))
        E = inputs.poisson_spheres(n, seed0 + b)
        lam, mu = inputs.lame_from_young(E, 0.3)
        lo, hi = inputs.lame_from_young(E.min(), 0.3), inputs.lame_from_young(E.max(), 0.3)
        cells.append((n, lam, mu, 0.5 * float(lo[0] + hi[0]), 0.5 * float(lo[1] + hi[1])))
    units = inputs.mandel_unit_strains()
    mandel = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    maxit = 20000
    groups = {}
    for i, c in enumerate(cells):
        groups.setdefault(c[0], []).append(i)
    order = sorted(groups.items())

    def sync_time(f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = f()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def ceff(sm, q):
        return np.stack([mandel * sm[6 * q + J] for J in range(6)], axis=1)

    def make(prec, warm, stream=None):
        hs = []
        for n, ix in order:
            systems = [(cells[i][1], cells[i][2], cells[i][3], cells[i][4]) for i in ix for J in range(6)]
            hs.append(lsfft.create_batch(systems, scheme="afb", prec=prec, f64_warmup=warm,
                                         stream=stream[n] if stream else None))
        return hs

    loads = [np.tile(units, (len(ix), 1)) for n, ix in order]
    out = {"cells": ncells, "sizes": {str(n): len(ix) for n, ix in order}}
    # FP64 group: the reference effective stiffness and iteration counts
    hs = make("f64", 0)
    (st, res), t64 = sync_time(lambda: lsfft.solve_group(hs, loads, tol, maxit))
    for h in hs:
        lsfft.destroy(h)
    ref, its64, vit64 = {}, {}, 0
    for (n, ix), (sm, it, r, sts) in zip(order, res):
        for q, i in enumerate(ix):
            ref[i] = ceff(sm, q)
            its64[i] = [int(v) for v in it[6 * q:6 * q + 6]]
            vit64 += n ** 3 * int(np.sum(it[6 * q:6 * q + 6]))
    converged = all(int(v) == lsfft.OK for (_, _, _, sts) in res for v in sts)
    out["group_f64"] = {"seconds": t64, "GVoxel_iter_per_s": vit64 / t64 / 1e9, "all_converged": converged,
                        "iters_mean": float(np.mean(list(its64.values()))),
                        "iters_max": int(np.max(list(its64.values())))}
    print(f"[bench] batched: FP64 group done ({t64:.2f} s)", file=sys.stderr, flush=True)
    # plain FP64 on a stratified subset of the cells
    t_plain, vit_plain, err_plain = 0.0, 0, 0.0
    subset = list(range(0, ncells, plain_stride))
    for i in subset:
        n, lam, mu, l0, m0 = cells[i]
        s = lsfft.Solver(lam, mu, l0, m0, scheme="afb", prec="f64")
        M = np.zeros((6, 6))
        for J in range(6):
            r, dt = sync_time(lambda: s.solve_device(units[J], tol=tol, maxit=maxit))
            t_plain += dt
            M[:, J] = mandel * r["sig_mean"]
            vit_plain += n ** 3 * r["iters"]
        s.close()
        err_plain = max(err_plain, float(np.linalg.norm(M - ref[i]) / np.linalg.norm(ref[i])))
    rate_plain = vit_plain / t_plain / 1e9
    t_plain_all = vit64 / (rate_plain * 1e9)
    out["plain_f64"] = {"cells_timed": len(subset), "seconds_timed": t_plain, "GVoxel_iter_per_s": rate_plain,
                        "seconds_for_all_cells": t_plain_all, "max_rel_err_ceff_vs_group_f64": err_plain}
    out["group_f64"]["speedup_over_plain_f64"] = t_plain_all / t64
    print(f"[bench] batched: plain FP64 on {len(subset)} cells done ({t_plain:.2f} s)", file=sys.stderr, flush=True)
    K = [int(max(max(its64[i]) for i in ix)) for n, ix in order]

    def score(res_list):
        err, vit = 0.0, 0
        for (n, ix), (sm, it, r, sts) in zip(order, res_list):
            vit += n ** 3 * int(np.sum(it))
            for q, i in enumerate(ix):
                err = max(err, float(np.linalg.norm(ceff(sm, q) - ref[i]) / np.linalg.norm(ref[i])))
        return err, vit

    # FP32 + warm start, one group graph over every size
    hs = make("f32", 5)
    (st, res), t32 = sync_time(lambda: lsfft.solve_group(hs, loads, 0.0, K))
    for h in hs:
        lsfft.destroy(h)
    err, vit = score(res)
    out["group_f32_warm5"] = {"seconds": t32, "GVoxel_iter_per_s": vit / t32 / 1e9,
                              "speedup_over_plain_f64": t_plain_all / t32, "speedup_over_group_f64": t64 / t32,
                              "max_rel_err_ceff_vs_group_f64": err}
    print(f"[bench] batched: FP32 group done ({t32:.2f} s)", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    # the same FP32 handles, one host thread and stream per size group
    streams = {n: torch.cuda.Stream() for n, ix in order}
    hs = make("f32", 5, streams)
    items = list(zip(hs, loads, K))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=len(items)) as pool:
        rs = list(pool.map(lambda it: lsfft.solve_batch(it[0], it[1], 0.0, it[2]), items))
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    for h in hs:
        lsfft.destroy(h)
    err, vit = score([(sm, it, r, sts) for (st, sm, it, r, sts) in rs])
    out["streams_f32_warm5"] = {"seconds": ts, "GVoxel_iter_per_s": vit / ts / 1e9, "streams": len(items),
                                "speedup_over_plain_f64": t_plain_all / ts, "max_rel_err_ceff_vs_group_f64": err}
    print(f"[bench] batched: FP32 streams done ({ts:.2f} s)", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    return out


def config_report():
    """Iterations to tolerance, status and wall time for the configurations of
    the paper's benchmark family: 16^3 BASIC FP64 (tol 1e-8); 64^3 at contrasts
    10 and 1e3, sharp and smooth interfaces, BASIC / FB / AFB, FP64 and FP32,
    six unit load cases -> Mandel C_eff (tol 1e-6); 256^3 AFB and DGO at
    contrasts 1e3 and 1e-3, PCD, eps_12 = 1e-3 (tol 1e-6).  GPU only; FP32
    C_eff is compared with the FP64 one."""
    import torch

    from paper_2009_03762_amd import inputs, lsfft
    r2 = np.sqrt(0.5)
    units = np.zeros((6, 6))
    for J in range(6):
        units[J, J] = 1.0 if J < 3 else r2   # unit Mandel norm, tensor components
    mandel = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])

    def cell(n, contrast, interface="sharp"):
        lam, mu = inputs.cubic_inclusion(n, n // 2, 1.0, contrast, 0.3, interface=interface, eps=1.0)
        l0, m0 = inputs.reference_medium_mean(1.0, contrast, 0.3)
        return lam, mu, l0, m0

    def timed(s, Eb, tol, maxit):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve_device(Eb, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    out = {}
    lam, mu, l0, m0 = cell(16, 10.0)
    s = lsfft.Solver(lam, mu, l0, m0, scheme="basic", prec="f64")
    r, dt = timed(s, inputs.macro_strain("11", 1e-3), 1e-8, 10000)
    s.close()
    out["16^3 basic f64 tol 1e-8"] = {"iters": r["iters"], "status": lsfft.status_string(r["status"]),
                                      "residual": r["residual"], "ms": dt * 1e3}
    print("[configs] 16^3 done", file=sys.stderr, flush=True)
    c2 = {}
    for contrast in (10.0, 1000.0):
        for interface in ("sharp", "smooth"):
            lam, mu, l0, m0 = cell(64, contrast, interface)
            ceff = {}
            for scheme in ("basic", "fb", "afb"):
                for prec in ("f64", "f32"):
                    s = lsfft.Solver(lam, mu, l0, m0, scheme=scheme, prec=prec)
                    M = np.zeros((6, 6))
                    its, sts, tot = [], [], 0.0
                    for J in range(6):
                        r, dt = timed(s, units[J], 1e-6, 20000)
                        M[:, J] = mandel * r["sig_mean"]
                        its.append(r["iters"])
                        sts.append(lsfft.status_string(r["status"]))
                        tot += dt
                    s.close()
                    ceff[(scheme, prec)] = M
                    ent = {"iters": its, "status": sorted(set(sts)), "ms_total": tot * 1e3,
                           "C1111": M[0, 0], "C1212_mandel": M[5, 5],
                           "asym": float(np.linalg.norm(M - M.T) / np.linalg.norm(M))}
                    if prec == "f32":
                        ent["rel_err_vs_f64"] = float(np.linalg.norm(M - ceff[(scheme, "f64")]) /
                                                      np.linalg.norm(ceff[(scheme, "f64")]))
                    c2[f"64^3 contrast {contrast:g} {interface} {scheme} {prec}"] = ent
            print(f"[configs] 64^3 contrast {contrast:g} {interface} done", file=sys.stderr, flush=True)
    out["config2"] = c2
    c3 = {}
    Eb = inputs.macro_strain("12", 1e-3)
    for contrast in (1e3, 1e-3):
        lam, mu, l0, m0 = cell(256, contrast)
        runs = [("afb f64", dict(scheme="afb", prec="f64")),
                ("afb f32 (5 fp64 warm-start iterations)", dict(scheme="afb", prec="f32", f64_warmup=5)),
                ("dgo p=1 M=4 f32", dict(scheme="dgo", prec="f32", dgo_images=4, dgo_weight_power=1)),
                ("dgo p=2 M=4 f32", dict(scheme="dgo", prec="f32", dgo_images=4, dgo_weight_power=2))]
        for name, kw in runs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = lsfft.Solver(lam, mu, l0, m0, disc="pcd", **kw)
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            r, dt = timed(s, Eb, 1e-6, 3000)
            s.close()
            c3[f"256^3 contrast {contrast:g} {name}"] = {
                "iters": r["iters"], "status": lsfft.status_string(r["status"]), "residual": r["residual"],
                "ms": dt * 1e3, "create_ms": setup * 1e3,
                "GVoxel_iter_per_s": 256 ** 3 * max(r["iters"], 1) / dt / 1e9}
            print(f"[configs] 256^3 {contrast:g} {name} done", file=sys.stderr, flush=True)
    out["config3"] = c3
    return out


def refine_study(n=256, tols=(1e-6, 1e-8), maxit=1500):
    """Wall time and iterations to a certified residual tolerance on the
    benchmark workload: F64, plain F32, F32 with the FP64 warm start, and
    F32 with FP64 iterative refinement (with and without warm-start
    iterations); each strain field is compared with a tight FP64 solution."""
    import torch

    from paper_2009_03762_amd import lsfft
    lam, mu, l0, m0, Eb = workload(n)
    shape = (6, n, n, n)
    ref = torch.zeros(shape, dtype=torch.float64, device="cuda")
    s = lsfft.Solver(lam, mu, l0, m0, scheme="afb", disc="pcd", prec="f64", form="displacement")
    r = s.solve_device(Eb, tol=1e-10, maxit=3000, eps_dev=ref)
    s.close()
    rn = torch.linalg.vector_norm(ref).item()
    out = {"reference": f"FP64 displacement form stopped at r = {r['residual']:.2e} after {r['iters']} iterations",
           "maxit": maxit, "runs": []}
    paths = (("f64", dict(prec="f64")), ("f32", dict(prec="f32")), ("f32_warm5", dict(prec="f32", f64_warmup=5)),
             ("f32_refine32", dict(prec="f32", refine=32)),
             ("f32_warm5_refine32", dict(prec="f32", refine=32, f64_warmup=5)),
             ("f32_warm20_refine16", dict(prec="f32", refine=16, f64_warmup=20)),
             ("f32_warm20_refine32", dict(prec="f32", refine=32, f64_warmup=20)))
    for tol in tols:
        for name, kw in paths:
            dt = torch.float64 if kw["prec"] == "f64" else torch.float32
            e = torch.zeros(shape, dtype=dt, device="cuda")
            s = lsfft.Solver(lam, mu, l0, m0, scheme="afb", disc="pcd", form="displacement", **kw)
            s.solve_device(Eb, tol=0.0, maxit=3, eps_dev=e)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = s.solve_device(Eb, tol=tol, maxit=maxit, eps_dev=e)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            err = (torch.linalg.vector_norm(e.double() - ref) / rn).item()
            s.close()
            del e
            row = {"tol": tol, "path": name, "status": int(o["status"]), "iters": int(o["iters"]),
                   "residual": float(o["residual"]), "ms": ms, "field_err": err}
            out["runs"].append(row)
            print(f"[bench] refine study {row}", file=sys.stderr, flush=True)
    del ref
    torch.cuda.synchronize()
    return out


def size_sweep(sizes=(32, 64, 128, 144, 192, 256, 288, 384, 512)):
    """Throughput of the benchmark workload (AFB, contrast 1e3, tol 0) across
    grid sizes, both precisions, automatic form, tuned schedule, replayed
    iteration graphs: where the path is launch-bound and where it streams."""
    import torch

    from paper_2009_03762_amd import lsfft
    out = []
    for n in sizes:
        lam, mu, l0, m0, Eb = workload(n)
        for prec in ("f32", "f64"):
            s = lsfft.Solver(lam, mu, l0, m0, scheme="afb", disc="pcd", prec=prec)
            sched, ms0, ms1 = lsfft.autotune(s.handle, 16)
            steps = int(max(20, min(800, 4e9 / n ** 3)))
            s.solve_device(Eb, tol=0.0, maxit=10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.solve_device(Eb, tol=0.0, maxit=steps)
            torch.cuda.synchronize()
            T = time.perf_counter() - t0
            # the strain form has no stencil (its schedule reports 0 planes)
            form = "displacement" if sched["stencil_planes"] > 0 else "strain"
            row = {"n": n, "prec": prec, "form": form, "steps": steps, "ms_per_iter": T / steps * 1e3,
                   "GVoxel_iter_per_s": n ** 3 * steps / T / 1e9, "schedule": sched}
            out.append(row)
            print(f"[bench] size sweep {row}", file=sys.stderr, flush=True)
            s.close()
            torch.cuda.empty_cache()
    return out


def oracle_timing(plan=((16, 100), (64, 10), (128, 4), (256, 1))):
    """The FP64 numpy oracle (its own FFT path) on one host core: seconds per
    iteration and GVoxel-iter/s of the benchmark cell at several sizes,
    `iters` full iterations each after setup."""
    out = []
    for n, iters in plan:
        r = cpu_baseline(n, iters)
        if "error" in r:
            out.append({"n": n, "error": r["error"]})
            continue
        out.append({"n": n, "iters": iters, "s_per_iter": n ** 3 / (r["value"] * 1e9),
                    "GVoxel_iter_per_s": r["value"], "cores": r["cores"]})
        print(f"[bench] oracle timing {out[-1]}", file=sys.stderr, flush=True)
    return {"host_cpus": os.cpu_count(), "runs": out}


def cpu_baseline(n=128, iters=8):
    """Time the oracle (as it stands) on the host: same cell at n^3, `iters`
    full iterations after setup, single-threaded numpy."""
    code = f"""
import time, json, sys
sys.path.insert(0, {ROOT!r})
from paper_2009_03762_amd import inputs
from oracle import solve3d
lam, mu = inputs.cubic_inclusion({n}, {n // 2}, 1.0, 1e3, 0.3)
l0, m0 = inputs.reference_medium_mean(1.0, 1e3, 0.3)
Eb = inputs.macro_strain('12', 1e-3)
ts = []
solve3d.solve_gfp(lam, mu, Eb, l0, m0, scheme='AFB', tol=0.0, maxit={iters}, disc='PCD',
                  callback=lambda k, e, T, r: ts.append(time.perf_counter()))
print(json.dumps({{"seconds": ts[-1] - ts[0], "iters": {iters}}}))
"""
    env = dict(os.environ)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[v] = "1"
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if out.returncode != 0:
        return {"error": out.stderr[-500:]}
    d = json.loads(out.stdout.strip().splitlines()[-1])
    return {
        "value": n ** 3 * d["iters"] / d["seconds"] / 1e9,
        "unit": "GVoxel-iter/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"FP64 numpy oracle, AFB fixed point on the same cubic-inclusion cell at {n}^3 "
                  f"(side {n // 2}, contrast 1e3), {d['iters']} full iterations timed after setup "
                  f"({d['seconds']:.1f} s), single thread",
    }


def copy_bandwidth(gib=1.0, reps=5):
    """Read + write GB/s of a plain device-to-device copy of `gib` GiB (after
    one untimed copy): the bandwidth a streaming kernel can reach here."""
    import torch
    n = int(gib * (1 << 30) // 4)
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del a, b
    return n * 4, 2 * n * 4 / dt / 1e9


def copy_probe(gib=1.0, reps=5):
    """A plain device-to-device copy of known size (calibrates HBM byte counters)."""
    nbytes, gbs = copy_bandwidth(gib, reps)
    print(json.dumps({"copy_bytes_each_way": nbytes, "reps": reps, "GBps_read_plus_write": gbs}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--prec", choices=["f32", "f64", "both"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-cells", type=int, default=48,
                    help="cells of the batched effective-stiffness measurement (48: the full set)")
    ap.add_argument("--configs", action="store_true",
                    help="instead of the bench line: iterations to tolerance for every configuration")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="instead of the bench line: the CPU oracle's speed at 16^3 to 256^3 (one core)")
    ap.add_argument("--size-sweep", action="store_true",
                    help="instead of the bench line: throughput from 32^3 to 512^3, both precisions")
    ap.add_argument("--refine-study", action="store_true",
                    help="instead of the bench line: time to a certified tolerance with FP64 refinement")
    ap.add_argument("--form", choices=["strain", "displacement"], default="displacement")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch schedule instead of the tuned one")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the solver is a "
              "single-GPU library; multi-GPU sharding is a design note, not an implemented path.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.configs:
        print(json.dumps(config_report()), flush=True)
        return
    if args.refine_study:
        print(json.dumps(refine_study(args.size)), flush=True)
        return
    if args.size_sweep:
        print(json.dumps(size_sweep()), flush=True)
        return
    if args.oracle_timing:
        print(json.dumps(oracle_timing()), flush=True)
        return
    tune = not args.no_autotune
    res32 = run_gpu("f32", args.size, args.steps, args.warmup, not args.no_breakdown, args.form, tune) \
        if args.prec in ("f32", "both") else None
    res64 = run_gpu("f64", args.size, args.steps, args.warmup, not args.no_breakdown, args.form, tune) \
        if args.prec in ("f64", "both") else None
    head = res32 if res32 is not None else res64
    line = {
        "metric": "GVoxel-iter/s, AFB fixed point 256^3 FP32 vs FP64; % HBM roofline",
        "value": head["value"],
        "unit": "GVoxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if res32 is not None else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.size}^3 cubic inclusion (side {args.size // 2}), E contrast 1e3, "
                               "nu 0.3, C0 = phase mean, eps_12 = 1e-3, PCD AFB, tol 0",
                   "grid": [args.size] * 3, "scheme": "AFB", "disc": "PCD", "form": args.form,
                   "reductions": "f64"},
        "roofline": head["roofline"],
        "whole_iteration_hbm_frac": head["whole_iteration_hbm_frac"],
        "whole_iteration_frac_fixed_balg": head["whole_iteration_frac_fixed_balg"],
        "bytes_per_voxel_iteration": head["bytes_per_voxel_iteration"],
        "kernels": head["kernels"],
        "autotune": head["autotune"],
    }
    # the same fractions against what a plain device copy reaches on this GPU
    _, copy_gbs = copy_bandwidth()
    line["copy_GBps"] = copy_gbs
    line["whole_iteration_frac_of_copy"] = head["whole_iteration_hbm_frac"] * HBM_PEAK_GBS / copy_gbs
    if head["roofline"] and head["roofline"].get("achieved"):
        line["roofline_frac_of_copy"] = head["roofline"]["achieved"] / copy_gbs
    if res32 is not None and res64 is not None:
        line["fp64"] = {k: res64[k] for k in ("value", "ms_per_step", "roofline", "whole_iteration_hbm_frac",
                                               "whole_iteration_frac_fixed_balg",
                                               "bytes_per_voxel_iteration", "kernels", "autotune")}
        line["fp32_speedup_over_fp64"] = res32["value"] / res64["value"]
    if not args.no_accuracy:
        line["equal_accuracy"] = equal_accuracy(args.size)
    if not args.no_batched and args.batched_cells > 0:
        line["batched_ceff"] = batched_ceff(args.batched_cells)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
