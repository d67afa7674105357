"""Benchmark: the whole hot path (H-matrix build, preconditioner setup and a
right-preconditioned GMRES solve to 1e-6) on the sphere + ellipsoid
workload (N = 20,000, lambda = 0.1, leaf <= 64, ACA 1e-4, RCM ordering,
fill-in tolerance 1e-2, one plane-wave right-hand side, GMRES(50)).

Prints one JSON line. `value` is whole-job RHS solves per second over the
timed steps (each step = build + setup + solve with inputs resident in HBM).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
PMC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_c2_sphere_ellipsoid_n20000.md")
KERNEL_SOURCES = ("paper_2111_13483_amd/csrc/kernels_sweep.hip", "paper_2111_13483_amd/csrc/kernels_solve.hip",
                  "paper_2111_13483_amd/csrc/kernels.h", "paper_2111_13483_amd/csrc/devcommon.h")
# the instrumented launches and their kernels' names
TIMING_EVERY = 4
KERNEL_NAME = {"sweep_fwd": "k_sweep_fwd", "sweep_bwd": "k_sweep_bwd", "near_mv": "k_near_mv", "far_mv": "k_far_mv"}
# the kernels behind each instrumented launch (the far matvec is two kernels,
# each dispatched once per matvec, on one stream inside one timed region)
PMC_KERNELS = {"sweep_fwd": ("k_sweep_fwd",), "sweep_bwd": ("k_sweep_bwd",), "near_mv": ("k_near_mv",),
               "far_mv": ("k_far_mv", "k_far_wave")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--n", type=int, default=0, help="override the point count (same structure)")
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work to sample")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--summarize-stats", metavar="DIR", help="summarise a rocprofv3 --stats run and exit")
    ap.add_argument("--out", help="summary file written by --summarize-*")
    ap.add_argument("--command", default="", help="command line recorded in the summary")
    ap.add_argument("--mixed", action="store_true",
                    help="mixed path: FP64 flexible GMRES(20) with inner GMRES(20) on complex64 copies")
    ap.add_argument("--batch", type=int, default=0, metavar="G",
                    help="batching run: G geometries of the many-geometry recipe, batched vs one-by-one setup")
    ap.add_argument("--batch-nmax", type=int, default=12000, help="largest N of the batching run")
    ap.add_argument("--serve", action="store_true",
                    help="serving run instead of the step benchmark: resident geometries, Poisson request arrivals")
    ap.add_argument("--serve-rates", default="5,20,80", help="request arrival rates per second")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="span of arrivals per rate")
    ap.add_argument("--write-workload", metavar="PATH",
                    help="write the workload (points, first right-hand side) for the hs_bench driver and exit")
    return ap.parse_args()


# ---------------------------------------------------------------- profile summaries

def _source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _find_csv(d, suffix):
    for base, _, files in os.walk(d):
        for f in sorted(files):
            if f.endswith(suffix):
                return os.path.join(base, f)
    raise SystemExit(f"no *{suffix} under {d}")


def _read_counters(d, counter):
    """Per-dispatch values of one counter: list of (kernel name, value)."""
    import csv
    rows = []
    with open(_find_csv(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") == counter:
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def _per_kernel(rows):
    agg = {}
    for name, v in rows:
        a = agg.setdefault(name, [0, 0.0])
        a[0] += 1
        a[1] += v
    return agg


def summarize_pmc(fetch_dir, write_dir, out, command, copy_bytes):
    fetch = _read_counters(fetch_dir, "FETCH_SIZE")
    write = _read_counters(write_dir, "WRITE_SIZE")
    # calibration: the largest copy dispatch (copy_bytes read and copy_bytes written)
    cf = max(v for n, v in fetch if "copy" in n.lower())
    cw = max(v for n, v in write if "copy" in n.lower())
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    af, aw = _per_kernel(fetch), _per_kernel(write)
    lines = ["# HBM traffic per launch, sphere + ellipsoid N = 20,000 (one step through the C-ABI driver hs_bench)",
             "",
             "Commands (FETCH_SIZE run, then WRITE_SIZE run):", "", "```", command, "```", "",
             f"Calibration: one device-to-device copy of {copy_bytes} bytes reads FETCH_SIZE = {cf:.0f} KiB and "
             f"WRITE_SIZE = {cw:.0f} KiB; scale factors {f_scale:.4f} (fetch) and {w_scale:.4f} (write).", "",
             "| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | scaled MB read | scaled MB written |",
             "|---|---|---|---|---|---|"]
    found = {}
    for key, pres in PMC_KERNELS.items():
        for pre in pres:
            names = [n for n in af if pre in n]
            if not names:
                continue
            nf = sum(af[n][0] for n in names)
            vf = sum(af[n][1] for n in names) / nf
            nw = sum(aw[n][0] for n in names if n in aw)
            vw = sum(aw[n][1] for n in names if n in aw) / max(nw, 1)
            rb, wb = vf * 1024.0 * f_scale, vw * 1024.0 * w_scale
            prb, pwb = found.get(key, (0.0, 0.0))
            found[key] = (prb + rb, pwb + wb)   # per launch: each kernel once
            lines.append(f"| {pre} | {nf} | {vf:.0f} | {vw:.0f} | {rb / 1e6:.1f} | {wb / 1e6:.1f} |")
    lines += ["", "Machine-readable (bench.py reads these while the kernel sources hash to `source`):", ""]
    for key, (rb, wb) in found.items():
        lines.append(f"traffic: kernel={key} read_bytes={rb:.0f} write_bytes={wb:.0f} source={_source_hash()}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_stats(d, out, command, top=25):
    import csv
    with open(_find_csv(d, "kernel_stats.csv")) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel time, sphere + ellipsoid N = 20,000 (bench.py default workload)", "",
             "Command:", "", "```", command, "```", "",
             "| kernel | calls | total ms | average us | min us | max us | share % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"]
        name = name if len(name) < 90 else name[:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def write_workload(args):
    """Binary workload for the C-ABI driver: header (n, k, self_h, leaf_max,
    restart, aca_tol, fill_tol, tol), points n x 3, one right-hand side."""
    import struct
    import workloads as W
    wl = W.make_config(args.workload, n=args.n or None, nrhs=1)
    if args.workload == "c2":
        wl.restart = 50
    with open(args.write_workload, "wb") as f:
        f.write(struct.pack("<qddiiddd", wl.n, wl.k, wl.self_h, wl.leaf_max, wl.restart, wl.aca_tol, wl.fill_tol,
                            wl.tol))
        f.write(np.ascontiguousarray(wl.points, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(wl.rhs[:, 0], dtype=np.complex128).tobytes())


def batch(args):
    """Batching: G geometries (sphere, ellipsoid, cube or plate; N uniform in
    [2000, nmax]; leaves 24-96; about ten points per wavelength), 4 plane-wave
    right-hand sides each. Times the H-matrix builds, the preconditioner
    setups once one by one and once batched (shared elimination launches),
    and the 4-column solves; progress goes to stderr."""
    import torch
    import paper_2111_13483_amd as hsl
    import workloads as W

    ctx = hsl.Context(0)
    geos = W.batch_geometries(args.batch, args.batch_nmax)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Hs = [hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol) for wl in geos]
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    print(f"batch: {len(Hs)} H-matrices in {t_build:.2f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    Ps1 = [hsl.Precond(ctx, H, "rcm", wl.fill_tol) for wl, H in zip(geos, Hs)]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    del Ps1
    print(f"batch: setups one by one {t_single:.2f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    Ps = hsl.Precond.many(ctx, Hs, "rcm", geos[0].fill_tol)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    print(f"batch: batched setup {t_batched:.2f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    iters, conv, cols = [], True, 0
    for wl, H, P in zip(geos, Hs, Ps):
        b = torch.as_tensor(np.ascontiguousarray(wl.rhs), device="cuda")
        x, st = hsl.solve(ctx, H, P, b, restart=wl.restart, tol=wl.tol)
        iters.append(max(s.iters for s in st))
        conv &= all(s.converged for s in st)
        cols += len(st)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    out = {"metric": "batched setup s and RHS solves/s over many geometries", "unit": "s, RHS/s",
           "data": "synthetic", "n_gpus": 1, "dtype": "c128",
           "config": {"workload": f"{len(geos)} geometries, N in [2000, {args.batch_nmax}], leaves 24-96, "
                                  "lambda = 10 h, 4 plane waves each, GMRES(30) to 1e-6",
                      "sum_n": int(sum(wl.n for wl in geos)),
                      "kinds": {k: sum(1 for wl in geos if wl.name == k) for k in ("sphere", "ellipsoid", "cube",
                                                                                   "plate")}},
           "h_build_s": t_build, "setup_one_by_one_s": t_single, "setup_batched_s": t_batched,
           "setup_speedup": t_single / t_batched, "solve_s": t_solve, "rhs_per_s": cols / t_solve,
           "iters_max": max(iters), "iters_median": float(np.median(iters)), "all_converged": conv}
    print(json.dumps(out), flush=True)


def serve(args):
    """Serving: four geometries resident on the GPU (admitted by device
    footprint); requests of 1-8 right-hand-side columns (half plane waves,
    half port vectors) arrive as a Poisson process and are batched per
    geometry, oldest request first, up to 16 columns per solve. Reports
    arrival-to-completion latency percentiles and RHS solves/s per rate;
    progress goes to stderr, one line per batch."""
    import torch
    import paper_2111_13483_amd as hsl
    import workloads as W

    ctx = hsl.Context(0)
    specs = [("c2", 8000), ("c2", 5000), ("c1", 4000), ("plate", 3000)]
    geos, t_setup = [], []
    srv = hsl.Server(ctx, 64 << 30, max_batch_cols=16, restart=50, tol=1e-6, max_iters=5000)
    for name, n in specs:
        wl = W.make_config(name, n=n)
        t0 = time.perf_counter()
        H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol)
        P = hsl.Precond(ctx, H, "rcm", wl.fill_tol)
        torch.cuda.synchronize()
        t_setup.append(time.perf_counter() - t0)
        geos.append((wl, srv.admit(H, P), H, P))
        print(f"serve: geometry {name} N={wl.n} ready in {t_setup[-1]:.2f} s", file=sys.stderr, flush=True)
    rng = np.random.default_rng(5)
    out = {"metric": "serving latency p50/p99 (arrival to completion) and RHS solves/s", "unit": "s, RHS/s",
           "data": "synthetic", "n_gpus": 1, "dtype": "c128",
           "config": {"workload": "resident " + ", ".join(f"{a} N={b}" for a, b in specs),
                      "columns_per_request": "uniform 1-8", "max_batch_cols": 16, "solver": "GMRES(50) to 1e-6"},
           "build_and_setup_s": t_setup, "rates": []}
    for rate in [float(r) for r in args.serve_rates.split(",")]:
        arr = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * args.serve_seconds * 3) + 8))
        arr = arr[arr <= args.serve_seconds]
        reqs = []
        for a in arr:
            gi = int(rng.integers(0, len(geos)))
            wl = geos[gi][0]
            nc = int(rng.integers(1, 9))
            cols = [W.plane_wave(wl.points, wl.k, rng) if rng.random() < 0.5 else W.port_vector(wl.n, rng)
                    for _ in range(nc)]
            reqs.append((a, gi, torch.as_tensor(np.stack(cols, axis=1), device="cuda")))
        torch.cuda.synchronize()
        t0 = hsl.Server.clock()
        ids, i, batches = [], 0, 0
        while i < len(reqs) or srv.pending()[0]:
            now = hsl.Server.clock() - t0
            while i < len(reqs) and reqs[i][0] <= now:
                ids.append(srv.submit(geos[reqs[i][1]][1], reqs[i][2], t0 + reqs[i][0]))
                i += 1
            if srv.pending()[0]:
                cols = srv.step()
                batches += 1
                print(f"serve: rate {rate:g} batch {batches} columns {cols} at {hsl.Server.clock() - t0:.2f} s",
                      file=sys.stderr, flush=True)
            elif i < len(reqs):
                time.sleep(max(0.0, reqs[i][0] - (hsl.Server.clock() - t0)))
        st = [srv.request(r) for r in ids]
        lat = np.array([s["t_done"] - s["t_arrival"] for s in st])
        ncol = sum(s["ncols"] for s in st)
        span = max(s["t_done"] for s in st) - t0
        out["rates"].append({"rate_per_s": rate, "requests": len(st), "columns": ncol, "batches": batches,
                             "latency_p50_s": float(np.percentile(lat, 50)),
                             "latency_p99_s": float(np.percentile(lat, 99)),
                             "rhs_per_s": ncol / span, "all_converged": all(s["converged"] for s in st),
                             "max_relres": max(s["relres"] for s in st)})
    print(json.dumps(out), flush=True)


def committed_traffic():
    """Scaled HBM bytes per launch from the committed counter summary; a
    kernel is absent when its sources changed since the counters were taken."""
    if not os.path.exists(PMC_SUMMARY):
        return {}
    src = _source_hash()
    out = {}
    with open(PMC_SUMMARY) as f:
        for line in f:
            if not line.startswith("traffic: "):
                continue
            kv = dict(p.split("=", 1) for p in line.split()[1:])
            if kv.get("source") == src:
                out[kv["kernel"]] = float(kv["read_bytes"]) + float(kv["write_bytes"])
    return out


def cpu_baseline(wl, gpu_iters, budget_s):
    """Time the oracle on a bounded sample of the same workload and scale each
    phase to the full problem (the oracle itself is not tuned for this)."""
    from oracle import aca as oaca
    from oracle import gmres as ogm  # noqa: F401
    from oracle import hmatrix as ohm
    from oracle import kernel as okern
    from oracle import ordering as oord
    from oracle import schur as osch
    from oracle import symbolic as osym

    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    hm = ohm.h_build(wl.points, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol, with_far=False)
    t_near = time.perf_counter() - t0
    far = hm.part.far
    nfar = len(far)
    # far ACA on a uniform random sample of blocks, scaled by the count
    t0 = time.perf_counter()
    idx = rng.permutation(nfar)
    done = 0
    far_s = []
    for b in idx:
        t, s = far[b]
        a0, a1 = hm.box_range(int(t))
        b0, b1 = hm.box_range(int(s))
        pt, ps = hm.pts[a0:a1], hm.pts[b0:b1]
        U, V, _, _ = oaca.aca(lambda i: okern.kernel_row(pt[i], ps, wl.k),
                              lambda j: okern.kernel_row(ps[j], pt, wl.k), a1 - a0, b1 - b0, wl.aca_tol)
        U, V = oaca.recompress(U, V, wl.aca_tol)
        far_s.append((b, U, V))
        done += 1
        if time.perf_counter() - t0 > 0.3 * budget_s:
            break
    t_far = (time.perf_counter() - t0) * nfar / done
    # setup: ordering + symbolic in full, elimination over the leading steps (flop-weighted)
    t0 = time.perf_counter()
    order = oord.make_order("rcm", hm.tree.nb, hm.part.near)
    sym = osym.symbolic(hm.tree.nb, hm.part.near, order)
    t_sym = time.perf_counter() - t0
    W, size = osch.initial_blocks(hm, sym)
    b = size.astype(float)
    flk = np.array([8 / 3 * b[k] ** 3 + sum(8 * b[k] ** 2 * b[j] for j in sym.rows[k])
                    + 8 * b[k] * 0.5 * (sum(b[j] for j in sym.rows[k]) ** 2 + sum(b[j] ** 2 for j in sym.rows[k]))
                    for k in range(sym.nb)])
    import scipy.linalg as sla
    t0 = time.perf_counter()
    kdone = 0
    for k in range(sym.nb):
        lu = sla.lu_factor(W[(k, k)])
        S = sym.rows[k]
        al = {j: -sla.lu_solve(lu, W[(k, j)]) for j in S}
        for a, i in enumerate(S):
            WT = W[(k, i)].T
            for j in S[a:]:
                key = (i, j)
                W[key] = W[key] + WT @ al[j]
        kdone = k + 1
        if time.perf_counter() - t0 > 0.3 * budget_s:
            break
    t_elim = (time.perf_counter() - t0) * flk.sum() / flk[:kdone].sum()
    # solve: one near+far matvec (far part scaled from the sample) and a
    # forward/backward sweep over the leading rows, per GMRES step
    v = rng.normal(size=hm.n) + 1j * rng.normal(size=hm.n)
    t0 = time.perf_counter()
    ohm.near_matvec(hm, v)
    t_nmv = time.perf_counter() - t0
    t0 = time.perf_counter()
    for bidx, U, V in far_s:
        t, s = far[bidx]
        a0, a1 = hm.box_range(int(t))
        b0, b1 = hm.box_range(int(s))
        _ = U @ (V @ v[b0:b1])
        _ = V.T @ (U.T @ v[a0:a1])
    t_fmv = (time.perf_counter() - t0) * nfar / max(len(far_s), 1)
    # the sweeps read each alpha block twice; time the dense products of the rows done above
    t0 = time.perf_counter()
    nrows = max(1, kdone)
    for k in range(nrows):
        for j in sym.rows[k]:
            A = W.get((k, j))
            if A is not None:
                _ = A.T @ v[:A.shape[0]]
                _ = A @ v[:A.shape[1]]
    t_sw = (time.perf_counter() - t0) * sym.nb / nrows
    t_iter = t_nmv + t_fmv + t_sw
    total = t_near + t_far + t_sym + t_elim + gpu_iters * t_iter
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": 1.0 / total, "unit": "RHS/s", "cores": threads, "kind": "oracle",
        "sample": (f"oracle on the same workload: near field in full, ACA on {done}/{nfar} far blocks, "
                   f"elimination over {kdone}/{sym.nb} steps (flop-weighted), one matvec + sweeps "
                   f"per GMRES step x {gpu_iters} steps; each phase scaled to the full problem"),
        "phase_s": {"h_build": t_near + t_far, "setup": t_sym + t_elim, "solve": gpu_iters * t_iter},
    }


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.out, args.command,
                      args.copy_calib_mib << 20)
        return
    if args.summarize_stats:
        summarize_stats(args.summarize_stats, args.out, args.command)
        return
    if args.write_workload:
        write_workload(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1"}))
        sys.exit(2)
    if args.serve:
        serve(args)
        return
    if args.batch:
        batch(args)
        return
    import torch
    import paper_2111_13483_amd as hsl
    import workloads as W

    wl = W.make_config(args.workload, n=args.n or None, nrhs=args.nrhs)
    if args.workload == "c2":
        wl.restart = 50
    dev = torch.device("cuda:0")
    ctx = hsl.Context(0)
    pts = torch.as_tensor(wl.points, device=dev)
    rhs = torch.as_tensor(np.ascontiguousarray(wl.rhs), device=dev)
    if args.copy_calib_mib:
        src = torch.ones(args.copy_calib_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        del src, dst
    torch.cuda.synchronize()

    def step(record):
        t0 = time.perf_counter()
        H = hsl.HMatrix(ctx, pts, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol, store_c64=args.mixed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P = hsl.Precond(ctx, H, "rcm", wl.fill_tol, mixed=args.mixed)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if args.mixed:
            x, st = hsl.solve(ctx, H, P, rhs if args.nrhs > 1 else rhs[:, 0], restart=20, tol=wl.tol, mixed=True,
                              inner_steps=20, inner_tol=1e-2)
        else:
            x, st = hsl.solve(ctx, H, P, rhs if args.nrhs > 1 else rhs[:, 0], restart=wl.restart, tol=wl.tol)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        record.append({"h_build": t1 - t0, "setup": t2 - t1, "solve": t3 - t2, "step": t3 - t0,
                       "iters": max(s.iters for s in st), "relres": max(s.relres for s in st),
                       "converged": all(s.converged for s in st)})
        return H, P

    warm = []
    for _ in range(args.warmup):
        step(warm)
    rec = []
    torch.cuda.synchronize()
    # kernel times from every TIMING_EVERY-th launch of each kernel inside
    # the timed steps: each bracketed launch adds ordering points to the
    # stream (about 11 ms per solve when every launch is bracketed)
    ctx.timing_begin(every=TIMING_EVERY)
    T0 = time.perf_counter()
    for _ in range(args.steps):
        H, P = step(rec)
    torch.cuda.synchronize()
    T = time.perf_counter() - T0
    ktimes = ctx.timing_end()
    hinfo, pinfo = H.info(), P.info()
    nrhs = args.nrhs
    steps = args.steps
    lat = np.array([r["step"] for r in rec])
    out = {
        "metric": "precond setup s + RHS solves/s at 1e-6 residual vs plain FP64; p50/p99 latency",
        "value": steps * nrhs / T,
        "unit": "RHS/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * T / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"{wl.name}: sphere+ellipsoid N={wl.n}, lambda=0.1, leaf<=64, ACA 1e-4, RCM, "
                               f"fill 1e-2, {nrhs} plane-wave RHS, GMRES({wl.restart}) to 1e-6",
                   "n": wl.n, "nrhs": nrhs,
                   "path": "mixed: FP64 FGMRES(20), inner GMRES(20) to 1e-2 on complex64 copies" if args.mixed
                   else "plain FP64"},
        "precond_setup_s": float(np.median([r["setup"] for r in rec])),
        "h_build_s": float(np.median([r["h_build"] for r in rec])),
        "solve_s": float(np.median([r["solve"] for r in rec])),
        "solve_rhs_per_s": nrhs / float(np.median([r["solve"] for r in rec])),
        "iters": rec[-1]["iters"], "relres": rec[-1]["relres"], "converged": rec[-1]["converged"],
        "vs_plain_fp64": 1.0,
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "hmatrix": {k: hinfo[k] for k in ("nb", "n_near", "n_far", "max_rank", "bytes_near", "bytes_far")},
        "precond": {k: pinfo[k] for k in ("n_pattern", "n_fill", "n_lowrank", "max_dk", "bytes_alpha", "bytes_d",
                                          "flops_setup")},
    }
    # algorithmic HBM bytes per launch: each stored matrix byte the kernel
    # needs is read once, plus one read and one write of its N x nrhs vectors
    vec = 32 * wl.n * nrhs
    alg = {"sweep_fwd": pinfo["bytes_alpha"] + vec,
           "sweep_bwd": pinfo["bytes_alpha"] + pinfo["bytes_d"] + vec,
           "near_mv": hinfo["bytes_near"] + vec,
           "far_mv": hinfo["bytes_far"] + vec}
    kern = {}
    for name, (cnt, ms) in ktimes.items():
        if cnt:
            avg = ms / cnt
            kern[name] = {"launches": cnt, "avg_ms": avg, "alg_bytes": alg[name],
                          "GB_per_s": alg[name] / (avg * 1e-3) / 1e9}
    # the near-field matvec runs on a second stream beside the far-field one:
    # its event time spans the concurrent far kernel, so it is reported but
    # not a candidate for the dominant kernel
    if "near_mv" in kern:
        kern["near_mv"]["overlaps"] = "far_mv"
    dom = max((k for k in kern if "overlaps" not in kern[k]), key=lambda k: kern[k]["launches"] * kern[k]["avg_ms"])
    traffic = committed_traffic()
    achieved = kern[dom]["GB_per_s"]
    out["roofline"] = {"bound": "hbm", "kernel": KERNEL_NAME[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic.get(dom),
                       "alg_bytes_per_launch": alg[dom], "avg_launch_ms": kern[dom]["avg_ms"]}
    out["kernels"] = kern
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, rec[-1]["iters"], args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
