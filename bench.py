#!/usr/bin/env python3
"""Benchmark: one time step's tridiagonal work on one MI355X.

Workload (synthetic, seeded, boundary-layer shaped; 2048 x 256 x 288 cells):
  * ADI momentum sweeps over u[Nz][Ny][Nx] (x fastest), FP64, PDD:
      x: lines of 2048, contiguous, P = 8, uniform mesh, r = dt*nu/dx^2
      y: lines of 256, stride Nx, P = 4, tanh-stretched wall-normal mesh
      z: lines of 288, stride Nx*Ny, periodic, P = 16
  * Poisson wavenumber solves, FP64, PPT, P = 4: spanwise rFFT of an N(0,1)
    field (input preparation, host, untimed) -> 145 x 256 x 2048 complex;
    k = 0 gauge pinned.
A step is the four solves in sequence, each one kernel launch (partition
factors, spikes and reduced-system rows are computed once, when the plans
are created).  Inputs are resident in HBM before timing; the solves run in
place, so each timed step solves the previous step's output (the work does
not depend on the values).

Prints one JSON line (metric, value = solved unknowns/s for the whole step,
roofline of the dominant kernel from HIP events, CPU-oracle baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NX, NY, NZ = 2048, 256, 288
HBM_PEAK_GBS = 8000.0
METRIC = "solved unknowns/s + % HBM peak; FP32+refine vs FP64 at 1e-12 rel err"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-refine", action="store_true", help="skip the FP32+refine measurement")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged eight-sub-grid batch")
    ap.add_argument("--no-independent", action="store_true", help="skip the independent-systems section")
    ap.add_argument("--no-pressure", action="store_true", help="skip the pressure-step (projection) section")
    ap.add_argument("--no-ns", action="store_true", help="skip the fractional-step time step section")
    ap.add_argument("--nx", type=int, default=NX)
    ap.add_argument("--ny", type=int, default=NY)
    ap.add_argument("--nz", type=int, default=NZ)
    return ap.parse_args()


def build_inputs(nx, ny, nz):
    import workloads as W
    t0 = time.perf_counter()
    u0 = W.cfg_field(nx, ny, nz, seed=0)
    phi0 = W.cfg_poisson_rhs(nx, ny, nz, seed=1)
    coef = {"x": W.momentum_uniform(nx), "y": W.momentum_stretched(ny), "z": W.momentum_periodic(nz)}
    ay, cy = W.poisson_metric(ny)
    lam = W.modified_wavenumbers(nz)
    log(f"inputs generated in {time.perf_counter() - t0:.1f}s")
    return u0, phi0, coef, ay, cy, lam


ITEMS = [  # name, direction, P, periodic, method
    ("adi_x", 0, 8, False, "PDD"),
    ("adi_y", 1, 4, False, "PDD"),
    # spanwise lines: 16 partitions of 18 rows (PDD drops entries ~1e-21 at
    # r = 0.083, so the result is the exact solution to round-off), which lets
    # the kernel run one 16-byte-access wavefront per partition
    ("adi_z", 2, 16, True, "PDD"),
    ("poisson", None, 4, False, "PPT"),
]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "the solves would shard as wall-normal slabs with PDD/PPT exchanges between neighbours, "
              "which one GPU cannot show", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1812_01178_amd as T

    nx, ny, nz = args.nx, args.ny, args.nz
    nk = nz // 2 + 1
    u0, phi0, coef, ay, cy, lam = build_inputs(nx, ny, nz)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = T.tri_create(0, stream.cuda_stream)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x)).cuda()
    du0, dphi0 = dev(u0), torch.as_tensor(phi0).cuda()
    u, phi = du0.clone(), dphi0.clone()
    dcoef = {k: tuple(dev(v) for v in abc) for k, abc in coef.items()}
    day, dcy, dlam = dev(ay), dev(cy), dev(lam)

    plans = {}
    for name, direction, P, per, meth in ITEMS:
        if name == "poisson":
            it = dict(kind=T.TRI_ITEM_POISSON, field=phi, Nx=nx, Ny=ny, Nz=nk, a=day, c=dcy, lam=dlam,
                      P=P, method=T.TRI_PPT)
        else:
            a, b, c = dcoef["xyz"[direction]]
            it = dict(kind=direction, field=u, Nx=nx, Ny=ny, Nz=nz, a=a, b=b, c=c, P=P,
                      periodic=int(per), method=T.TRI_PDD if meth == "PDD" else T.TRI_PPT)
        plans[name] = T.tri_plan_create(ctx, [it])
        log(f"plan {name}: {T.tri_plan_item_describe(plans[name], 0)}")
    T.tri_sync_status(ctx)

    unknowns = {"adi_x": nx * ny * nz, "adi_y": nx * ny * nz, "adi_z": nx * ny * nz,
                "poisson": nk * ny * nx}
    bytes_per = {"adi_x": 16, "adi_y": 16, "adi_z": 16, "poisson": 32}   # read d + write x, FP64

    # ---------------- self-check on sampled lines, pristine inputs ---------
    # backward error of each solve (needs no reference solution; the oracle
    # parity of these shapes is in the GPU tests)
    residual = {}
    if not args.no_parity:
        residual = sampled_residuals(T, plans, u, phi, du0, dphi0, u0, phi0, coef, ay, cy, lam, ITEMS,
                                     np.random.default_rng(123))
        for name, r in residual.items():
            log(f"residual {name}: max line backward error {r:.2e}")
        u.copy_(du0)
        phi.copy_(dphi0)
        torch.cuda.synchronize()
    # every solve's result on the pristine input, kept on the host for the
    # comparison with the oracle in the CPU-baseline leg (outside any timing)
    keep = args.cpu_seconds > 0 and not args.no_parity
    pristine = {"fp64": pristine_outputs(plans, u, phi, du0, dphi0, ITEMS, T)} if keep else {}

    # ---------------- timed steps -----------------------------------------
    names = [it[0] for it in ITEMS]

    def step(events=None):
        for idx, name in enumerate(names):
            if events is not None:
                events[idx].record(stream)
            T.tri_plan_execute(plans[name])
        if events is not None:
            events[len(names)].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T.tri_sync_status(ctx)
    per_item_ms = {n: float(np.mean([ev[s][i].elapsed_time(ev[s][i + 1]) for s in range(args.steps)]))
                   for i, n in enumerate(names)}
    step_ms_events = float(np.mean([ev[s][0].elapsed_time(ev[s][-1]) for s in range(args.steps)]))
    ms_per_step = wall * 1e3 / args.steps
    total_unknowns = sum(unknowns.values())
    value = total_unknowns / (ms_per_step * 1e-3)
    kernels = {}
    for n in names:
        gbs = unknowns[n] * bytes_per[n] / (per_item_ms[n] * 1e-3) / 1e9
        kernels[n] = {"ms": round(per_item_ms[n], 4), "unknowns": unknowns[n],
                      "alg_bytes": unknowns[n] * bytes_per[n], "GB_s": round(gbs, 1),
                      "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                      "unknowns_per_s": unknowns[n] / (per_item_ms[n] * 1e-3)}
        log(f"{n}: {per_item_ms[n]:.4f} ms  {gbs:.0f} GB/s  ({100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s)")
    for i, n in enumerate(names):
        kernels[n]["ms_median"] = round(float(np.median([ev[s][i].elapsed_time(ev[s][i + 1])
                                                         for s in range(args.steps)])), 4)
    dom = max(names, key=lambda n: per_item_ms[n])
    step_bytes = sum(unknowns[n] * bytes_per[n] for n in names)

    # ---------------- copy ceiling: the library's reference copy ----------
    # (u <- du0 moves the same 16 B per unknown as a solve of the field)
    copy = copy_ceiling(T, ctx, stream, u, du0, max(args.steps, 20))
    for n in names:
        kernels[n]["copy_frac"] = round(kernels[n]["GB_s"] / copy["GB_s"], 4)
    log(f"reference copy: {copy['GB_s']:.0f} GB/s ({copy['bytes'] / 1e9:.3f} GB per call); "
        + ", ".join(f"{n} {100 * kernels[n]['copy_frac']:.1f}%" for n in names) + " of it")

    # ---------------- FP32 elimination + FP64 refinement -----------------
    refine = None
    if not args.no_refine:
        refine = refine_section(T, ctx, stream, u, phi, du0, dphi0, dcoef, day, dcy, dlam, coef,
                                u0, phi0, ay, cy, lam, nx, ny, nz, nk, args, unknowns, bytes_per, per_item_ms,
                                pristine if keep else None)

    # ---------------- ragged batch: eight sub-grids in one plan -----------
    ragged = None
    if not args.no_ragged:
        del u, phi, du0, dphi0
        torch.cuda.empty_cache()
        ragged = ragged_section(T, ctx, stream, args, pristine if keep else None)

    # ---------------- pressure step: FFT + Poisson + correction -----------
    pressure = None
    if not args.no_pressure:
        pressure = pressure_section(T, ctx, stream, args, nx, ny, nz, copy["GB_s"])
        pressure["three_d"] = pressure3d_section(T, ctx, stream, args, nx, ny, nz, copy["GB_s"])

    # ---------------- the whole fractional-step time step -----------------
    fractional = None
    if not args.no_ns:
        fractional = fractional_step_section(T, ctx, stream, args, nx, ny, nz)

    # ---------------- independent systems with their own coefficients -----
    independent = None
    if not args.no_independent:
        independent = independent_section(T, ctx, stream, args, pristine if keep else None)

    # ---------------- CPU oracle baseline (bounded sample) ----------------
    # and, outside every timed region, each result's error against the oracle
    cpu = None
    oracle_err = None
    if args.cpu_seconds > 0:
        import oracle      # the CPU-baseline leg is the only use of the oracle here
        cpu = cpu_baseline(oracle, u0, phi0, coef, ay, cy, lam, args.cpu_seconds)
        if keep:
            oracle_err = oracle_parity(oracle, pristine, u0, phi0, coef, ay, cy, lam)
            if refine is not None:
                refine["oracle_err_max_line"] = oracle_err.pop("fp32_refine")
            if ragged is not None:
                for prec_name in ("fp64", "fp32_refine"):
                    ragged[prec_name]["oracle_err_max_line"] = oracle_err.pop("ragged_" + prec_name)
            if independent is not None:
                for name, e in oracle_err.pop("independent").items():
                    independent[name]["oracle_err_max_line"] = e
            oracle_err = oracle_err["fp64"]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ADI x/y/z (PDD) + Poisson wavenumber (PPT) solves on {nx}x{ny}x{nz}",
                   "Nx": nx, "Ny": ny, "Nz": nz, "Nk": nk,
                   "P": {n: it[2] for n, it in zip(names, ITEMS)},
                   "method": {n: it[4] for n, it in zip(names, ITEMS)},
                   "unknowns_per_step": total_unknowns,
                   "launch": {n: T.tri_plan_item_describe(plans[n], 0) for n in names}},
        "hbm_frac_step": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_ms_events": step_ms_events,
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kernels[dom]["GB_s"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(kernels[dom]["GB_s"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, T.tri_plan_item_describe(plans[dom], 0)),
                     "copy_GB_s": copy["GB_s"], "copy_frac": kernels[dom]["copy_frac"]},
        "copy_ceiling": copy,
        "residual_max_line": residual,
        "oracle_err_max_line": oracle_err,
        "oracle_err_def": ("per line max_j |x - x_oracle| / max_j |x_oracle| on the pristine input, worst line, "
                           "against the FP64 oracle: PDD/PPT at the FP64 run's P (PDD exact to round-off there), "
                           "the same solve for FP32+refine; ragged: per sub-grid, the composed x -> y -> z step "
                           "and the Poisson solves"),
        "fp32_refine": refine,
        "ragged_batch": ragged,
        "pressure_step": pressure,
        "fractional_step": fractional,
        "independent_systems": independent,
        "cpu_baseline": cpu,
    }
    for p in plans.values():
        T.tri_plan_destroy(p)
    T.tri_destroy(ctx)
    print(json.dumps(out), flush=True)


def pristine_outputs(plans, u, phi, du0, dphi0, items, T):
    """Each item's plan run once from the pristine input; its whole result
    copied to the host (the field is restored afterwards)."""
    out = {}
    for name, *_ in items:
        if name == "poisson":
            phi.copy_(dphi0)
            T.tri_plan_execute(plans[name])
            out[name] = phi.cpu().numpy()
        else:
            u.copy_(du0)
            T.tri_plan_execute(plans[name])
            out[name] = u.cpu().numpy()
    u.copy_(du0)
    phi.copy_(dphi0)
    return out


def line_relerr(got, ref, axis):
    """Worst per-line relative error max_j |x - x_ref| / max_j |x_ref| along `axis`."""
    num = np.max(np.abs(got - ref), axis=axis)
    den = np.max(np.abs(ref), axis=axis)
    return float(np.max(num / np.where(den == 0, 1.0, den)))


def oracle_parity(oracle, pristine, u0, phi0, coef, ay, cy, lam):
    """Every result kept from a pristine-input run against the FP64 oracle, line
    by line (the CPU-baseline leg; nothing here is timed).  FP64 PDD/PPT against
    the oracle at the same P.  FP32+refine converges to A^-1 d, so it is held to
    the same oracle solve: PDD at the benchmark's P drops entries below 1e-15
    (1e-21 for the spanwise lines), so the oracle's PDD is the exact solution to
    round-off, and the Poisson reference is the oracle's PPT (exact)."""
    t0 = time.perf_counter()
    err = {}
    for name, d, P, per, meth in ITEMS:
        if name == "poisson":
            ref = np.array(phi0, copy=True)
            oracle.poisson(ref, ay, cy, lam, P=P)
            axis = 1
        else:
            ref = np.array(u0, copy=True)
            oracle.adi_sweep(oracle.PDD, d, ref, *coef["xyz"[d]], P, per)
            axis = 2 - d
        for prec in ("fp64", "fp32_refine"):
            if prec in pristine:
                e = line_relerr(pristine[prec].pop(name), ref, axis)
                err.setdefault(prec, {})[name] = e
                log(f"oracle parity {prec} {name}: worst line {e:.2e}")
        del ref
    for prec in ("fp64", "fp32_refine"):
        pristine.pop(prec, None)
    refs = {}
    for prec in ("fp64", "fp32_refine"):
        key = "ragged_" + prec
        if key not in pristine:
            continue
        worst_adi = worst_poi = 0.0
        for s_, g in enumerate(pristine.pop(key)):
            if s_ not in refs:
                # the FP64 plan's partition counts (PDD admitted only where it is exact to round-off)
                cf = dict(zip("xyz", g["coef"]))
                ref = np.array(g["u0"], copy=True)
                for d in range(3):
                    oracle.adi_sweep(oracle.PDD, d, ref, *cf["xyz"[d]], g["P"][d], d == 2)
                pref = np.array(g["phi0"], copy=True)
                oracle.poisson(pref, *g["metric"], g["lam"], P=g["P"][3])
                refs[s_] = (ref, pref)
            ref, pref = refs[s_]
            worst_adi = max(worst_adi, line_relerr(g["u"], ref, 0))
            worst_poi = max(worst_poi, line_relerr(g["phi"], pref, 1))
        err[key] = {"adi_step": worst_adi, "poisson": worst_poi}
        log(f"oracle parity ragged {prec}: ADI step {worst_adi:.2e}, Poisson {worst_poi:.2e}")
    if "independent" in pristine:
        ind = pristine.pop("independent")
        r, d, P = ind["r"], ind["d"], ind["P"]
        n, nlines = d.shape
        e = {}
        for name, method in (("pdd_fp64", oracle.PDD), ("ppt_fp64", oracle.PPT), ("ppt_fp32_refine", oracle.PPT)):
            if name not in ind:
                continue
            ref = np.array(d, copy=True).ravel()
            oracle.solve_batch(method, ref, n, nlines, 1, s_j=nlines, s_b0=1, s_b1=0, a=-r, b=1 + 2 * r, c=-r,
                               cs_j=0, cs_b0=1, cs_b1=0, P=P)
            e[name] = line_relerr(ind[name], ref.reshape(n, nlines), 0)
            log(f"oracle parity independent {name}: worst line {e[name]:.2e}")
        err["independent"] = e
    log(f"oracle parity of every kept result: {time.perf_counter() - t0:.1f}s")
    return err


def sampled_lines(u, u0, direction, nsamp, rng):
    """(result, input) of nsamp random lines along `direction` of a [Nz][Ny][Nx] field,
    as (nsamp, n) arrays."""
    import torch
    nz, ny, nx = u0.shape
    if direction == 0:
        j, k = rng.integers(0, ny, nsamp), rng.integers(0, nz, nsamp)
        return u[torch.as_tensor(k), torch.as_tensor(j), :].cpu().numpy(), u0[k, j, :]
    if direction == 1:
        i, k = rng.integers(0, nx, nsamp), rng.integers(0, nz, nsamp)
        return u[torch.as_tensor(k), :, torch.as_tensor(i)].cpu().numpy(), u0[k, :, i]
    i, j = rng.integers(0, nx, nsamp), rng.integers(0, ny, nsamp)
    return u[:, torch.as_tensor(j), torch.as_tensor(i)].T.cpu().numpy(), u0[:, j, i].T


def sampled_residuals(T, plans, u, phi, du0, dphi0, u0, phi0, coef, ay, cy, lam, items, rng):
    """Run each item's plan once from the pristine input and return the largest per-line
    backward error over sampled lines (48 per sweep; 24 Poisson lines including the
    modes 0, 1, 2 and the last)."""
    out = {}
    nk = phi0.shape[0]
    nx = phi0.shape[2]
    for name, direction, P, per, meth in items:
        if name == "poisson":
            phi.copy_(dphi0)
            T.tri_plan_execute(plans[name])
            ks = rng.integers(0, nk, 24)
            ks[:4] = [0, 1, 2, nk - 1]
            iis = rng.integers(0, nx, 24)
            import torch
            got = phi[torch.as_tensor(ks), :, torch.as_tensor(iis)].cpu().numpy()
            d = phi0[ks, :, iis].copy()
            a, b, c, pin = poisson_rows(ay, cy, lam[ks])
            d[pin, 0] = 0.0
            out[name] = line_residual(a, b, c, got, d)
        else:
            u.copy_(du0)
            T.tri_plan_execute(plans[name])
            got, lines = sampled_lines(u, u0, direction, 48, rng)
            a, b, c = coef["xyz"[direction]]
            out[name] = line_residual(a, b, c, got, lines, per)
    return out


def apply_tri(a, b, c, x, axis=-1, periodic=False):
    """(A x, |a x_{j-1}| + |b x_j| + |c x_{j+1}|) along `axis` of x, FP64 (numpy).  The
    coefficients are 1-D along the row axis, or (axis = -1) any shape that broadcasts
    against x; the ends couple through a_0 and c_{n-1} only when periodic."""
    x = np.moveaxis(x, axis, -1)
    xm, xp = np.roll(x, 1, -1), np.roll(x, -1, -1)
    if not periodic:
        xm[..., 0] = 0.0
        xp[..., -1] = 0.0
    t0, t1, t2 = a * xm, b * x, c * xp
    return (np.moveaxis(t0 + t1 + t2, -1, axis),
            np.moveaxis(np.abs(t0) + np.abs(t1) + np.abs(t2), -1, axis))


def apply_tri_dev(a, b, c, x, dim, periodic):
    """A x along dimension `dim` of a device tensor x (torch, FP64); a, b, c are 1-D
    device tensors along `dim`; the ends couple only when periodic."""
    import torch
    shape = [1] * x.dim()
    shape[dim] = -1
    xm, xp = torch.roll(x, 1, dim), torch.roll(x, -1, dim)
    if not periodic:
        xm.select(dim, 0).zero_()
        xp.select(dim, -1).zero_()
    return a.view(shape) * xm + b.view(shape) * x + c.view(shape) * xp


def line_residual(a, b, c, x, d, periodic=False):
    """Largest per-line backward error max_j |d - A x| / max_j (|a x_{j-1}| + |b x_j| + |c x_{j+1}|)
    over lines along the last axis of x and d (a self-check of a solve that needs no reference
    solution; a correct FP64 solve gives ~1e-16)."""
    ax, scale = apply_tri(a, b, c, x, -1, periodic)
    r = np.max(np.abs(d - ax), axis=-1)
    s_ = np.max(scale, axis=-1)
    return float(np.max(r / np.where(s_ == 0, 1.0, s_)))


def poisson_rows(ay, cy, lam_k):
    """Coefficient rows (a, b, c) of the wavenumber systems for the modes lam_k (one row
    per mode), with the gauge-pinned row 0 (x_0 = 0) where lam_k == 0."""
    n = ay.size
    a = np.broadcast_to(ay, (lam_k.size, n)).copy()
    c = np.broadcast_to(cy, (lam_k.size, n)).copy()
    b = -(ay + cy)[None, :] - lam_k[:, None]
    pin = lam_k == 0.0
    b[pin, 0] = 1.0
    c[pin, 0] = 0.0
    a[pin, 0] = 0.0
    return a, b, c, pin


def copy_ceiling(T, ctx, stream, dst, src, reps):
    """Median rate of the library's reference copy (tri_stream_copy) of the
    whole field, read + write bytes per second, HIP events on the context
    stream."""
    import torch
    n = src.numel()
    for _ in range(3):
        T.tri_stream_copy(ctx, dst, src, n)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        T.tri_stream_copy(ctx, dst, src, n)
        b.record(stream)
    torch.cuda.synchronize()
    T.tri_sync_status(ctx)
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    nbytes = 2 * n * 8
    return {"kernel": "tri_stream_copy (one pass, 16-byte non-temporal loads and stores)",
            "bytes": nbytes, "ms_median": round(ms, 4), "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_2048x256x288.md")
KERNEL_SOURCES = {"strided": ["tri_kernels.hip"], "contiguous-reg": ["tri_contig_reg.hip"],
                  "contiguous-staged": ["tri_kernels.hip"]}


def source_digest(kind):
    """sha256 over the files a kernel kind is compiled from (its source and the shared headers)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1812_01178_amd", "csrc")
    for f in KERNEL_SOURCES[kind] + ["tri_device.h", "tri_internal.h"]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(item, launch):
    """HBM bytes per launch of `item` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the summary was taken for another launch shape or before the
    kernel's sources last changed."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    kind = launch.split()[0]
    if kind not in KERNEL_SOURCES:
        return None
    for ln in lines:
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0] == item:
            recorded_launch, digest, total_gb = cells[1].strip("`"), cells[2].strip("`"), cells[-2]
            if recorded_launch != launch or digest != source_digest(kind):
                return None
            try:
                return float(total_gb) * 1e9
            except ValueError:
                return None
    return None


REFINE_P = {"adi_y": 8, "adi_z": 8}


def refine_section(T, ctx, stream, u, phi, du0, dphi0, dcoef, day, dcy, dlam, coef, u0, phi0,
                   ay, cy, lam, nx, ny, nz, nk, args, unknowns, bytes_per, fp64_ms, pristine=None):
    """FP32 elimination + FP64 residual refinement (Poisson modes k <= 2 in
    FP64) on the step's four solves, timed like the FP64 step; the backward
    error of sampled lines is checked (the refined result is the exact
    solution, so it is ~1e-16 like an FP64 solve)."""
    import torch
    # the refined result is the exact solution whatever the inner solver's
    # partition count; the refinement kernel takes up to 16 wavefronts of up
    # to 16 rows or up to 8 wavefronts of up to 40 rows, and the wall-normal
    # and spanwise lines run fastest at P = 8 (16-row and 36-row chunks)
    items = [(nm, d, REFINE_P.get(nm, P), per, meth) for nm, d, P, per, meth in ITEMS]
    plans, descr = {}, {}
    for name, direction, P, per, meth in items:
        if name == "poisson":
            it = dict(kind=T.TRI_ITEM_POISSON, field=phi, Nx=nx, Ny=ny, Nz=nk, a=day, c=dcy, lam=dlam, P=P,
                      method=T.TRI_PPT)
        else:
            a, b, c = dcoef["xyz"[direction]]
            it = dict(kind=direction, field=u, Nx=nx, Ny=ny, Nz=nz, a=a, b=b, c=c, P=P, periodic=int(per),
                      method=T.TRI_PDD)
        plans[name] = T.tri_plan_create(ctx, [it], prec=T.TRI_F32_REFINE)
        descr[name] = T.tri_plan_item_describe(plans[name], 0)
        log(f"refine plan {name}: {descr[name]}")
    err = sampled_residuals(T, plans, u, phi, du0, dphi0, u0, phi0, coef, ay, cy, lam, items,
                            np.random.default_rng(321))
    for name, r in err.items():
        log(f"refine residual {name}: max line backward error {r:.2e}")
    try:
        T.tri_sync_status(ctx)
        status = "converged"
    except T.TriError as ex:
        status = str(ex)
    if pristine is not None:
        pristine["fp32_refine"] = pristine_outputs(plans, u, phi, du0, dphi0, items, T)
    u.copy_(du0)
    phi.copy_(dphi0)
    torch.cuda.synchronize()
    names = [it[0] for it in items]
    for _ in range(args.warmup):
        for n_ in names:
            T.tri_plan_execute(plans[n_])
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(args.steps)]
    for s_ in range(args.steps):
        for i_, n_ in enumerate(names):
            ev[s_][i_].record(stream)
            T.tri_plan_execute(plans[n_])
        ev[s_][len(names)].record(stream)
    torch.cuda.synchronize()
    try:
        T.tri_sync_status(ctx)
    except T.TriError:
        pass   # timed steps re-solve their own output; convergence was checked above
    out = {"kernels": {}, "residual_max_line": err, "status": status}
    tot_r = tot_64 = 0.0
    for i_, n_ in enumerate(names):
        ms = float(np.mean([ev[s_][i_].elapsed_time(ev[s_][i_ + 1]) for s_ in range(args.steps)]))
        gbs = unknowns[n_] * bytes_per[n_] / (ms * 1e-3) / 1e9
        out["kernels"][n_] = {"ms": round(ms, 4), "GB_s": round(gbs, 1), "launch": descr[n_],
                              "fp64_ms": round(fp64_ms[n_], 4), "speedup_vs_fp64": round(fp64_ms[n_] / ms, 3)}
        tot_r += ms
        tot_64 += fp64_ms[n_]
        log(f"refine {n_}: {ms:.4f} ms ({gbs:.0f} GB/s) vs FP64 {fp64_ms[n_]:.4f} ms")
    # the FP64 path at the refined solves' partition counts where they differ
    # (same configuration; timing only, the FP64 step keeps its own counts)
    for name, direction, P, per, meth in items:
        P64 = next(p_ for nm, _, p_, _, _ in ITEMS if nm == name)
        if P == P64:
            continue
        a, b, c = dcoef["xyz"[direction]]
        plan64 = T.tri_plan_create(ctx, [dict(kind=direction, field=u, Nx=nx, Ny=ny, Nz=nz, a=a, b=b, c=c, P=P,
                                              periodic=int(per), method=T.TRI_PDD)])
        for _ in range(args.warmup):
            T.tri_plan_execute(plan64)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            T.tri_plan_execute(plan64)
        e1.record(stream)
        torch.cuda.synchronize()
        ms64 = e0.elapsed_time(e1) / args.steps
        T.tri_plan_destroy(plan64)
        k_ = out["kernels"][name]
        k_["fp64_ms_same_P"] = round(ms64, 4)
        k_["speedup_vs_fp64_same_P"] = round(ms64 / k_["ms"], 3)
        log(f"refine {name}: FP64 at the same P = {P}: {ms64:.4f} ms")
    u.copy_(du0)
    torch.cuda.synchronize()
    out["ms_step"] = round(tot_r, 4)
    out["fp64_ms_step"] = round(tot_64, 4)
    out["unknowns_per_s"] = sum(unknowns[n_] for n_ in names) / (tot_r * 1e-3)
    out["speedup_vs_fp64"] = round(tot_64 / tot_r, 3)
    for p_ in plans.values():
        T.tri_plan_destroy(p_)
    return out


def pressure_section(T, ctx, stream, args, nx, ny, nz, copy_gbs):
    """The projection that ends a fractional sub-step (Sec. 2.2) on the
    benchmark grid: divergence of (v, w) fused into the spanwise real FFT,
    the Poisson wavenumber solves (PPT, P = 4, plan), inverse FFT fused with
    the spanwise gradient correction, wall-normal gradient correction.
    v[Nz][Ny+1][Nx] (walls zero) and w[Nz][Ny][Nx] are N(0,1) from torch's
    device generator (seed 0).  Checked before timing: the corrected
    velocity is divergence free to round-off (plain torch ops on the
    device)."""
    import torch
    import workloads as W
    nk = nz // 2 + 1
    dy = np.diff(W.tanh_faces(ny))
    dz = 1.0 / nz
    ay, cy = W.poisson_metric(ny)
    lam = W.modified_wavenumbers(nz)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x)).cuda()
    ddy, day, dcy, dlam = dev(dy), dev(ay), dev(cy), dev(lam)
    g = torch.Generator(device="cuda").manual_seed(0)
    v = torch.randn((nz, ny + 1, nx), dtype=torch.float64, device="cuda", generator=g)
    v[:, 0, :] = 0.0
    v[:, ny, :] = 0.0
    w = torch.randn((nz, ny, nx), dtype=torch.float64, device="cuda", generator=g)
    ph = torch.empty((nk, ny, nx), dtype=torch.complex128, device="cuda")
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    plan = T.tri_plan_create(ctx, [dict(kind=T.TRI_ITEM_POISSON, field=ph, Nx=nx, Ny=ny, Nz=nk, a=day, c=dcy,
                                        lam=dlam, P=4, method=T.TRI_PPT)])
    log(f"pressure plan: {T.tri_plan_item_describe(plan, 0)}")

    def div(vv, ww):
        return (vv[:, 1:, :] - vv[:, :-1, :]) / ddy[None, :, None] + (torch.roll(ww, -1, 0) - ww) / dz

    parts = ["divergence_rfft", "poisson", "correct"]

    def step(events=None):
        fns = (lambda: T.projection_divergence_rfft(ctx, v, w, ddy, dz, ph),
               lambda: T.tri_plan_execute(plan),
               lambda: T.projection_correct(ctx, ph, phi, v, w, ddy, dz))
        for i, fn in enumerate(fns):
            if events is not None:
                events[i].record(stream)
            fn()
        if events is not None:
            events[3].record(stream)

    # self-check on the pristine field: the corrected velocity must be
    # divergence free to round-off (the oracle parity is in the GPU tests)
    div0 = div(v, w).abs().max().item()
    step()
    T.tri_sync_status(ctx)
    div1 = div(v, w).abs().max().item()
    log(f"pressure step: max |div| {div0:.3e} -> {div1:.3e} ({div1 / div0:.1e})")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        step(ev[s_])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T.tri_sync_status(ctx)
    T.tri_plan_destroy(plan)
    cells = nx * ny * nz
    alg = {"divergence_rfft": 8 * nz * (ny + 1) * nx + 8 * cells + 16 * nk * ny * nx,
           "poisson": 32 * nk * ny * nx,
           "correct": 16 * nk * ny * nx + 8 * cells + 16 * cells + 8 * cells + 16 * nz * (ny - 1) * nx}
    kernels = {}
    for i, n in enumerate(parts):
        ms = float(np.mean([ev[s_][i].elapsed_time(ev[s_][i + 1]) for s_ in range(args.steps)]))
        gbs = alg[n] / (ms * 1e-3) / 1e9
        kernels[n] = {"ms": round(ms, 4), "alg_bytes": alg[n], "GB_s": round(gbs, 1),
                      "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "copy_frac": round(gbs / copy_gbs, 4)}
        log(f"pressure {n}: {ms:.4f} ms  {gbs:.0f} GB/s  ({100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s, "
            f"{100 * gbs / copy_gbs:.1f}% of the reference copy)")
    ms_step = wall * 1e3 / args.steps
    total = sum(alg.values())
    out = {"grid": [nx, ny, nz], "P": 4, "ms_per_step": round(ms_step, 4), "alg_bytes": total,
           "GB_s": round(total / (ms_step * 1e-3) / 1e9, 1),
           "hbm_frac": round(total / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "cells_per_s": cells / (ms_step * 1e-3), "kernels": kernels,
           "divergence_before": div0, "divergence_after": div1, "divergence_ratio": div1 / div0}
    log(f"pressure step: {ms_step:.3f} ms, {out['GB_s']:.0f} GB/s over the step, "
        f"{cells / (ms_step * 1e-3) / 1e9:.1f} G cells/s")
    del v, w, ph, phi
    torch.cuda.empty_cache()
    return out


def pressure3d_section(T, ctx, stream, args, nx, ny, nz, copy_gbs):
    """The 3-D projection (walls at both x-ends as well): divergence of
    (u, v, w) fused into the spanwise FFT, streamwise cosine transform, the
    shifted wall-normal solves (one matrix per (k, i), PPT, P = 8: at most
    32 rows per partition on the fly), inverse cosine transform, inverse FFT
    with the w correction, v and u corrections.  u[Nz][Ny][Nx+1] (x-end
    faces zero), v, w as in the spanwise-only step, N(0,1) from torch's device
    generator (seed 1).  Checked before timing: divergence free to round-off."""
    import torch
    import workloads as W
    nk = nz // 2 + 1
    P = 8
    dy = np.diff(W.tanh_faces(ny))
    dx, dz = 1.0 / nx, 1.0 / nz
    ay, cy = W.poisson_metric(ny)
    lamz = W.modified_wavenumbers(nz)
    lamx = (4.0 / dx ** 2) * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x)).cuda()
    ddy, day, dcy, dlz, dlx = dev(dy), dev(ay), dev(cy), dev(lamz), dev(lamx)
    g = torch.Generator(device="cuda").manual_seed(1)
    u = torch.randn((nz, ny, nx + 1), dtype=torch.float64, device="cuda", generator=g)
    u[:, :, 0] = 0.0
    u[:, :, nx] = 0.0
    v = torch.randn((nz, ny + 1, nx), dtype=torch.float64, device="cuda", generator=g)
    v[:, 0, :] = 0.0
    v[:, ny, :] = 0.0
    w = torch.randn((nz, ny, nx), dtype=torch.float64, device="cuda", generator=g)
    ph = torch.empty((nk, ny, nx), dtype=torch.complex128, device="cuda")
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")

    def div(uu, vv, ww):
        return ((uu[:, :, 1:] - uu[:, :, :-1]) / dx + ((vv[:, 1:, :] - vv[:, :-1, :]) / ddy[None, :, None]
                + (torch.roll(ww, -1, 0) - ww) / dz))

    parts = ["divergence_rfft", "dct", "poisson_shifted", "idct", "correct"]
    fns = (lambda: T.projection3d_divergence_rfft(ctx, u, v, w, dx, ddy, dz, ph),
           lambda: T.streamwise_dct(ctx, ph),
           lambda: T.poisson_shifted_solve(ctx, ph, day, dcy, dlz, dlx, P=P, method=T.TRI_PPT),
           lambda: T.streamwise_idct(ctx, ph),
           lambda: T.projection3d_correct(ctx, ph, phi, u, v, w, dx, ddy, dz))

    def step(events=None):
        for i, fn in enumerate(fns):
            if events is not None:
                events[i].record(stream)
            fn()
        if events is not None:
            events[len(fns)].record(stream)

    div0 = div(u, v, w).abs().max().item()
    step()
    T.tri_sync_status(ctx)
    div1 = div(u, v, w).abs().max().item()
    log(f"pressure 3-D: max |div| {div0:.3e} -> {div1:.3e} ({div1 / div0:.1e})")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(fns) + 1)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        step(ev[s_])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T.tri_sync_status(ctx)
    cells = nx * ny * nz
    spec = 16 * nk * ny * nx
    alg = {"divergence_rfft": 8 * nz * ny * (nx + 1) + 8 * nz * (ny + 1) * nx + 8 * cells + spec,
           "dct": 2 * spec, "poisson_shifted": 2 * spec, "idct": 2 * spec,
           # spectrum in, phi out, w read + write, phi read once for the u and v corrections
           "correct": spec + 8 * cells + 16 * cells + 8 * cells + 16 * nz * (ny - 1) * nx
                      + 16 * nz * ny * (nx - 1)}
    kernels = {}
    for i, n in enumerate(parts):
        ms = float(np.mean([ev[s_][i].elapsed_time(ev[s_][i + 1]) for s_ in range(args.steps)]))
        gbs = alg[n] / (ms * 1e-3) / 1e9
        kernels[n] = {"ms": round(ms, 4), "alg_bytes": alg[n], "GB_s": round(gbs, 1),
                      "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "copy_frac": round(gbs / copy_gbs, 4)}
        log(f"pressure 3-D {n}: {ms:.4f} ms  {gbs:.0f} GB/s  ({100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s)")
    ms_step = wall * 1e3 / args.steps
    total = sum(alg.values())
    out = {"grid": [nx, ny, nz], "P": P, "ms_per_step": round(ms_step, 4), "alg_bytes": total,
           "GB_s": round(total / (ms_step * 1e-3) / 1e9, 1),
           "hbm_frac": round(total / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "cells_per_s": cells / (ms_step * 1e-3), "kernels": kernels,
           "divergence_before": div0, "divergence_after": div1, "divergence_ratio": div1 / div0}
    log(f"pressure 3-D step: {ms_step:.3f} ms, {out['GB_s']:.0f} GB/s over the step")
    del u, v, w, ph, phi
    torch.cuda.empty_cache()
    return out


# Table 1 of the paper (4 Tesla P100, FP64): wall-clock seconds per time step
# (three sub-steps) for two of its grids, as context only
PAPER_TABLE1 = [{"grid": [1024, 256, 512], "s_per_step": 2.60, "hardware": "4x Tesla P100"},
                {"grid": [2048, 256, 1024], "s_per_step": 7.74, "hardware": "4x Tesla P100"}]


def fractional_step_section(T, ctx, stream, args, nx, ny, nz):
    """The whole fractional-step time step (ns_step: three Runge-Kutta sub-steps,
    each the momentum right-hand side, nine PDD sweeps (x, y, z of u, v, w at
    P = 8, 4, 16; the velocity update fused into the z sweeps' stores), the
    3-D projection with PPT shifted solves at P = 8, the pressure update) on
    the benchmark grid, dt = 1e-3, nu = 1e-3, from a random state (N(0,1)/10
    from torch's device generator, seed 4, wall faces zero).  Checked before
    timing: one step leaves the velocity divergence free to round-off.  The
    oracle parity of the step is in the GPU tests (grids up to 256 x 64 x 48
    and 48 x 16 x 144)."""
    import torch
    import workloads as W
    dx, dz = 1.0 / nx, 1.0 / nz
    dy = np.diff(W.tanh_faces(ny))
    ddy = torch.as_tensor(dy).cuda()
    g = torch.Generator(device="cuda").manual_seed(4)
    u = 0.1 * torch.randn((nz, ny, nx + 1), dtype=torch.float64, device="cuda", generator=g)
    u[:, :, 0] = 0.0
    u[:, :, nx] = 0.0
    v = 0.1 * torch.randn((nz, ny + 1, nx), dtype=torch.float64, device="cuda", generator=g)
    v[:, 0, :] = 0.0
    v[:, ny, :] = 0.0
    w = 0.1 * torch.randn((nz, ny, nx), dtype=torch.float64, device="cuda", generator=g)
    p = torch.zeros((nz, ny, nx), dtype=torch.float64, device="cuda")

    def div():
        return ((u[:, :, 1:] - u[:, :, :-1]) / dx + (v[:, 1:, :] - v[:, :-1, :]) / ddy[None, :, None]
                + (torch.roll(w, -1, 0) - w) / dz).abs().max().item()
    P_adi, P_poi = (8, 4, 16), 8
    t0 = time.perf_counter()
    ns = T.ns_create(ctx, nx, ny, nz, dx, dz, dy, 1e-3, 1e-3, P_adi, P_poi)
    create_s = time.perf_counter() - t0
    try:
        d0 = div()
        T.ns_step(ns, u, v, w, p, ctx)
        T.tri_sync_status(ctx)
        d1 = div()
        log(f"fractional step: max |div| {d0:.3e} -> {d1:.3e} ({d1 / d0:.1e})")
        for _ in range(args.warmup):
            T.ns_step(ns, u, v, w, p, ctx)
        torch.cuda.synchronize()
        steps = max(3, args.steps // 4)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            T.ns_step(ns, u, v, w, p, ctx)
        e1.record(stream)
        torch.cuda.synchronize()
        T.tri_sync_status(ctx)
        ms = e0.elapsed_time(e1) / steps
        finite = bool(torch.isfinite(u).all() and torch.isfinite(v).all() and torch.isfinite(w).all())
    finally:
        T.ns_destroy(ns)
    cells = nx * ny * nz
    out = {"grid": [nx, ny, nz], "P_adi": list(P_adi), "P_poisson": P_poi, "dt": 1e-3, "nu": 1e-3,
           "ms_per_step": round(ms, 3), "steps": steps, "cells_per_s": cells / (ms * 1e-3),
           "plan_create_s": round(create_s, 2), "divergence_before": d0, "divergence_after_first_step": d1,
           "divergence_ratio": d1 / d0, "finite": finite,
           "paper_table1_context": [dict(r, cells_per_s=r["grid"][0] * r["grid"][1] * r["grid"][2] / r["s_per_step"])
                                    for r in PAPER_TABLE1]}
    log(f"fractional step: {ms:.2f} ms per time step (3 sub-steps), {cells / (ms * 1e-3) / 1e9:.2f} G cells/s; "
        f"Table 1 context: 1024x256x512 in 2.60 s, 2048x256x1024 in 7.74 s on 4 P100")
    del u, v, w, p
    torch.cuda.empty_cache()
    return out


def independent_section(T, ctx, stream, args, pristine=None):
    """4096 independent systems of 64 unknowns, a = c = -r, b = 1 + 2r with one
    r ~ U[0.1, 10] per system, d ~ U[-1, 1] (seed 0), P = 4, lines side by side
    (row j of system s at j * 4096 + s): FP64 PDD and PPT and FP32 + refinement
    (PPT inner solver), each checked by the backward error of every system
    (PDD's is its truncation: PDD is exact only where the dropped reduced-system
    entries vanish, and r up to 10 with 16 rows per partition leaves them near
    3e-3).  The problem is 2 MB, so the times are launch-level, not bandwidth
    figures."""
    import torch
    import workloads as W
    n, nlines, P = 64, 4096, 4
    r, dl = W.cfg_independent(nlines, n, seed=0)
    d = np.ascontiguousarray(dl.T)
    a, b, c = -r, 1 + 2 * r, -r
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x)).cuda()
    da, db, dc, d0 = dev(a), dev(b), dev(c), dev(d)
    lines = (n, nlines, 1, nlines, 1, 0)
    out = {"systems": nlines, "n": n, "P": P, "unknowns": n * nlines}
    for name, fn, prec in (("pdd_fp64", T.tri_pdd_solve, T.TRI_F64),
                           ("ppt_fp64", T.tri_ppt_solve, T.TRI_F64),
                           ("ppt_fp32_refine", T.tri_ppt_solve, T.TRI_F32_REFINE)):
        x = d0.clone()
        info = fn(ctx, da, db, dc, x, lines, coef_strides=(0, 1, 0), P=P, prec=prec, info=True)
        T.tri_sync_status(ctx)
        got = x.cpu().numpy()
        if pristine is not None:
            pristine.setdefault("independent", {"r": r, "d": d, "P": P})[name] = got
        reps = 50
        for _ in range(3):
            fn(ctx, da, db, dc, x, lines, coef_strides=(0, 1, 0), P=P, prec=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn(ctx, da, db, dc, x, lines, coef_strides=(0, 1, 0), P=P, prec=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        # systems are columns: row j of system s at [j][s]
        res = {"us_per_solve": round(us, 2), "unknowns_per_s": n * nlines / (us * 1e-6),
               "residual_max_line": line_residual(a[:, None], b[:, None], c[:, None], got.T, d.T)}
        if prec == T.TRI_F32_REFINE:
            res["sweeps"] = info["sweeps"]
        out[name] = res
        log(f"independent {name}: {us:.1f} us per solve, backward error {res['residual_max_line']:.2e}")
    return out


def ragged_section(T, ctx, stream, args, pristine=None):
    """The batched ragged workload: eight sub-grids (Nx, Ny, Nz) covering
    Nx in {256..2048}, Ny in {128, 256}, Nz in {96, 288}, each with an x, y and
    periodic-z momentum sweep (PDD) and its Poisson wavenumber solves (PPT),
    all in one plan with P = 0 (the plan times P in {1,2,4,8,16}; PDD only
    where its dropped entries are <= 1e-15).  FP64: every solve of a
    dependency level in one launch of the level kernel (three launches a
    step); the step is also timed as a HIP graph, with the strided solves of
    one kernel instance batched instead, without batching, and in FP32 +
    refinement (strided refinement solves of one instance batched).  Every sub-grid's result is
    checked by its backward error (the oracle parity of this batch is in the
    GPU tests)."""
    import torch
    import workloads as W
    t0 = time.perf_counter()
    grids = []
    for s_, (nx, ny, nz) in enumerate(W.RAGGED_SUBGRIDS):
        grids.append(dict(shape=(nx, ny, nz), u0=W.cfg_field(nx, ny, nz, seed=200 + s_),
                          phi0=W.cfg_poisson_rhs(nx, ny, nz, seed=300 + s_),
                          coef=(W.momentum_uniform(nx), W.momentum_stretched(ny), W.momentum_periodic(nz)),
                          metric=W.poisson_metric(ny), lam=W.modified_wavenumbers(nz)))
    log(f"ragged inputs generated in {time.perf_counter() - t0:.1f}s")
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x)).cuda()
    keep = []
    for g in grids:
        g["du0"], g["dphi0"] = dev(g["u0"]), torch.as_tensor(g["phi0"]).cuda()
        g["u"], g["phi"] = g["du0"].clone(), g["dphi0"].clone()
        g["dcoef"] = [tuple(dev(v) for v in c) for c in g["coef"]]
        g["dmetric"] = tuple(dev(v) for v in g["metric"])
        g["dlam"] = dev(g["lam"])

    def items():
        out = []
        for g in grids:
            nx, ny, nz = g["shape"]
            for d in range(3):
                a, b, c = g["dcoef"][d]
                out.append(dict(kind=d, field=g["u"], Nx=nx, Ny=ny, Nz=nz, a=a, b=b, c=c, P=0,
                                periodic=int(d == 2), method=T.TRI_PDD))
            out.append(dict(kind=T.TRI_ITEM_POISSON, field=g["phi"], Nx=nx, Ny=ny, Nz=nz // 2 + 1,
                            a=g["dmetric"][0], c=g["dmetric"][1], lam=g["dlam"], P=0, method=T.TRI_PPT))
        return out

    def reset():
        for g in grids:
            g["u"].copy_(g["du0"])
            g["phi"].copy_(g["dphi0"])
        torch.cuda.synchronize()

    def ragged_residual(g):
        """Backward errors of one sub-grid's ADI step and Poisson solves (plain torch
        ops in FP64 on the device)."""
        u = g["u"]
        y, s_ = u, u.abs()
        for d, dim in ((2, 0), (1, 1), (0, 2)):   # A_x A_y A_z u: apply z first
            a, b, c = g["dcoef"][d]
            y = apply_tri_dev(a, b, c, y, dim, d == 2)
            s_ = apply_tri_dev(a.abs(), b.abs(), c.abs(), s_, dim, d == 2)
        e_adi = ((y - g["du0"]).abs().max() / s_.max()).item()
        ay, cy = g["dmetric"]
        lam = g["dlam"]
        pin = lam == 0
        a = ay.view(1, -1, 1)
        b = (-(ay + cy)).view(1, -1, 1) - lam.view(-1, 1, 1)
        c = cy.view(1, -1, 1).expand(lam.numel(), -1, 1).clone()
        b[pin, 0, 0] = 1.0
        c[pin, 0, 0] = 0.0
        rhs = g["dphi0"].clone()
        rhs[pin, 0, :] = 0.0
        x = g["phi"]
        xm, xp = torch.roll(x, 1, 1), torch.roll(x, -1, 1)
        xm[:, 0, :] = 0.0
        xp[:, -1, :] = 0.0
        t0, t1, t2 = a * xm, b * x, c * xp
        r = (rhs - (t0 + t1 + t2)).abs().amax(dim=1)
        sc = (t0.abs() + t1.abs() + t2.abs()).amax(dim=1)
        e_poi = (r / torch.where(sc == 0, torch.ones_like(sc), sc)).max().item()
        return e_adi, e_poi

    def timed(run, steps):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    unknowns = sum(3 * nx * ny * nz + (nz // 2 + 1) * ny * nx for nx, ny, nz in W.RAGGED_SUBGRIDS)
    alg_bytes = sum(3 * 16 * nx * ny * nz + 32 * (nz // 2 + 1) * ny * nx for nx, ny, nz in W.RAGGED_SUBGRIDS)
    out = {"subgrids": W.RAGGED_SUBGRIDS, "unknowns_per_step": unknowns, "alg_bytes_per_step": alg_bytes}
    for prec_name, prec in (("fp64", T.TRI_F64), ("fp32_refine", T.TRI_F32_REFINE)):
        t0 = time.perf_counter()
        plan = T.tri_plan_create(ctx, items(), prec=prec)
        create_s = time.perf_counter() - t0
        n_items = 4 * len(grids)
        Ps = [T.tri_plan_item_partitions(plan, i) for i in range(n_items)]
        descr = [T.tri_plan_item_describe(plan, i) for i in range(n_items)]
        batches = sorted({d.split(k)[1].split()[0] for d in descr for k in ("batch=", "level=") if k in d})
        n_launch = T.tri_plan_launch_count(plan)
        mode = "one launch per dependency level" if any("level=" in d for d in descr) else \
            "strided solves of one kernel instance batched"
        reset()
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
        if pristine is not None:
            pristine["ragged_" + prec_name] = [
                dict(shape=g["shape"], u0=g["u0"], phi0=g["phi0"], coef=g["coef"], metric=g["metric"], lam=g["lam"],
                     P=Ps[4 * s_:4 * s_ + 4], u=g["u"].cpu().numpy(), phi=g["phi"].cpu().numpy())
                for s_, g in enumerate(grids)]
        errs = [ragged_residual(grids[s_]) for s_ in (range(len(grids)) if prec == T.TRI_F64 else (0, 3, 4))]
        parity = max(max(e) for e in errs)
        # in-place solves re-solve their own output; each field is reset
        # before a timed series (a Poisson mode repeatedly solved grows or
        # shrinks by its condition number per step)
        reset()
        ms = timed(lambda: T.tri_plan_execute(plan), args.steps)
        T.tri_plan_capture(plan)
        reset()
        ms_graph = timed(lambda: T.tri_plan_graph_launch(plan), args.steps)
        try:
            T.tri_sync_status(ctx)
            status = "ok"
        except T.TriError as ex:
            status = str(ex)
        T.tri_plan_destroy(plan)
        res = {"ms_per_step": round(ms, 4), "ms_per_step_graph": round(ms_graph, 4),
               "unknowns_per_s": unknowns / (ms * 1e-3), "unknowns_per_s_graph": unknowns / (ms_graph * 1e-3),
               "hbm_frac_graph": round(alg_bytes / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "P": Ps, "batched_launches": len(batches), "plan_create_s": round(create_s, 2),
               "residual_max": parity, "status": status,
               "residual": "per sub-grid: the step x -> y -> z solves A_z A_y A_x u = u0, so "
                           "max|A_x A_y A_z u - u0| / max(|A_x| |A_y| |A_z| |u|), and the largest "
                           "per-line backward error of the Poisson solves"}
        res["launches_per_step"] = n_launch
        res["launch_mode"] = mode
        os.environ["TRI_BATCH"] = "0"
        plan = T.tri_plan_create(ctx, items(), prec=prec)
        os.environ.pop("TRI_BATCH")
        reset()
        res["ms_per_step_unbatched"] = round(timed(lambda: T.tri_plan_execute(plan), args.steps), 4)
        res["launches_per_step_unbatched"] = T.tri_plan_launch_count(plan)
        T.tri_plan_destroy(plan)
        if prec == T.TRI_F64:
            # the alternative grouping: strided solves of one kernel instance
            # batched, every other solve in a launch of its own kernel (with
            # that grouping's own partition-count and shape choices)
            os.environ["TRI_BATCH"] = "1"
            plan = T.tri_plan_create(ctx, items(), prec=prec)
            os.environ.pop("TRI_BATCH")
            reset()
            T.tri_plan_execute(plan)
            T.tri_sync_status(ctx)
            pi_err = max(max(ragged_residual(g)) for g in grids)
            reset()
            pi_ms = timed(lambda: T.tri_plan_execute(plan), args.steps)
            T.tri_plan_capture(plan)
            reset()
            pi_graph = timed(lambda: T.tri_plan_graph_launch(plan), args.steps)
            res["per_instance_batches"] = {
                "ms_per_step": round(pi_ms, 4), "ms_per_step_graph": round(pi_graph, 4),
                "unknowns_per_s_graph": unknowns / (pi_graph * 1e-3),
                "launches_per_step": T.tri_plan_launch_count(plan),
                "P": [T.tri_plan_item_partitions(plan, i) for i in range(n_items)],
                "residual_max": pi_err}
            T.tri_plan_destroy(plan)
            log(f"ragged {prec_name} per-instance batches: {pi_ms:.3f} ms/step ({pi_graph:.3f} ms as graph), "
                f"{res['per_instance_batches']['launches_per_step']} launches, residual {pi_err:.2e}")
        out[prec_name] = res
        log(f"ragged {prec_name}: {ms:.3f} ms/step ({ms_graph:.3f} ms as graph), "
            f"{unknowns / (ms_graph * 1e-3) / 1e9:.1f} G unknowns/s, {n_launch} launches ({mode}), "
            f"residual {parity:.2e}, P={Ps}")
    out["refine_speedup_vs_fp64"] = round(out["fp64"]["ms_per_step_graph"] / out["fp32_refine"]["ms_per_step_graph"], 3)
    return out


def cpu_baseline(oracle, u0, phi0, coef, ay, cy, lam, target_s):
    """The oracle as it stands, all host cores, on a sample of each solve's
    lines (every q-th outer index), scaled to unknowns/s of the whole step."""
    cores = len(os.sched_getaffinity(0))
    Nz, Ny, Nx = u0.shape
    Nk = phi0.shape[0]

    def run(frac_outer, threads=cores):
        t_item, n_item = {}, {}
        # x lines: sample z-planes
        qz = max(1, int(round(1 / frac_outer)))
        sub = np.array(u0[::qz], copy=True, order="C")     # the inputs stay pristine
        t0 = time.perf_counter()
        oracle.adi_sweep(oracle.PDD, 0, sub, *coef["x"], ITEMS[0][2], False, nthreads=threads)
        t_item["adi_x"], n_item["adi_x"] = time.perf_counter() - t0, sub.size
        sub = np.array(u0[::qz], copy=True, order="C")
        t0 = time.perf_counter()
        oracle.adi_sweep(oracle.PDD, 1, sub, *coef["y"], ITEMS[1][2], False, nthreads=threads)
        t_item["adi_y"], n_item["adi_y"] = time.perf_counter() - t0, sub.size
        qy = max(1, int(round(1 / frac_outer)))
        sub = np.array(u0[:, ::qy], copy=True, order="C")
        t0 = time.perf_counter()
        oracle.adi_sweep(oracle.PDD, 2, sub, *coef["z"], ITEMS[2][2], True, nthreads=threads)
        t_item["adi_z"], n_item["adi_z"] = time.perf_counter() - t0, sub.size
        qk = max(1, int(round(1 / frac_outer)))
        sub = np.array(phi0[::qk], copy=True, order="C")
        t0 = time.perf_counter()
        oracle.poisson(sub, ay, cy, lam[::qk], P=ITEMS[3][2], nthreads=threads)
        t_item["poisson"], n_item["poisson"] = time.perf_counter() - t0, sub.size
        return t_item, n_item

    frac = 1 / 64
    t_item, n_item = run(frac)
    spent = sum(t_item.values())
    if spent < target_s / 4:
        frac = min(1.0, frac * target_s / max(spent, 1e-3))
        t_item, n_item = run(frac)
    full = {"adi_x": Nx * Ny * Nz, "adi_y": Nx * Ny * Nz, "adi_z": Nx * Ny * Nz, "poisson": Nk * Ny * Nx}
    step_s = sum(t_item[k] / n_item[k] * full[k] for k in full)
    total = sum(full.values())
    log(f"cpu oracle: {sum(t_item.values()):.1f}s on {sum(n_item.values())} unknowns, "
        f"{cores} threads -> full step {step_s:.2f}s")
    # one thread, on a sample sized for about 3 s (perfect scaling assumed)
    spent = sum(t_item.values())
    frac1 = max(1 / 288, min(frac, 3.0 * frac / max(spent * cores, 1e-3)))
    t1, n1 = run(min(1.0, frac1), threads=1)
    step1_s = sum(t1[k] / n1[k] * full[k] for k in full)
    log(f"cpu oracle, 1 thread: {sum(t1.values()):.1f}s on {sum(n1.values())} unknowns -> full step {step1_s:.1f}s")
    return {"value": total / step_s, "unit": "unknowns/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle PDD/PPT (FP64, C, OpenMP {cores} threads) on {planes(frac)} of each of the "
                      f"4 solves ({sum(n_item.values())} unknowns, {sum(t_item.values()):.1f}s), scaled to the step",
            "step_seconds_est": step_s, "cpu_model": cpu_model(),
            "one_thread": {"value": total / step1_s, "unit": "unknowns/s",
                           "sample": f"{planes(min(1.0, frac1))} ({sum(n1.values())} unknowns, "
                                     f"{sum(t1.values()):.1f}s), scaled to the step"}}


def planes(frac):
    q = int(round(1 / frac))
    return "every outer plane" if q == 1 else f"every {q}th outer plane"


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
