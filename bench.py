"""Benchmark of the FOSB hot path on one MI355X.

One step = one pass of the whole hot path over the workload "mixed_k5":
unit icosphere levels s = 2..5 (480 / 1920 / 7680 / 30720 RWG), k = 5,
plane wave d = e_z, p = e_x, radial Gaussian covariance (sigma 0.01, ell 0.5),
combination technique L0 = 2, L = 5 (4 level pairs), 181 angles in the
xz-plane:
  EFIE assembly of every level -> LU + first moment + RHS weights of every
  level -> RHS correlation and two-sided solve of every CT pair -> far-field
  variance.
Inputs (meshes, uploaded tables) and output buffers are resident on the GPU
before the timed region.  The metric is level-pair solves per second of the
mixed-precision path (FP32-complex MFMA LU + FP64 refinement); the FP64 path
is timed too and reported next to it, with the relative difference of the two
variances.  Refinement stops once the estimated relative error of the
solves (from the decay of the corrections) is below --ir-tol (default 1e-8);
the reported mixed-vs-FP64 difference confirms the accuracy reached.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision both|mixed|fp64]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "mixed": 157.3}          # dense MFMA TFLOP/s (FP64, FP32)
HBM_PEAK = 8000.0                               # GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_k_gemm_f32_mixed_k5.txt")
# the kernel's source and the factorisation that sets its launch shapes
GEMM_SRC = [os.path.join(ROOT, "paper_2308_01457_amd", "csrc", f) for f in ("gemm.hip", "lu.hip")]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, or None when it is missing or the kernel's source or the
    factorisation that shapes its launches has changed since the counters were
    taken."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in GEMM_SRC)).hexdigest()
        if kv.get("source_sha256") != sha:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--max-level", type=int, default=5)
    ap.add_argument("--ir-tol", type=float, default=1e-7,
                    help="mixed path: target relative error of the refined solves (an order below the 1e-6 "
                         "agreement with the FP64 path that the metric asks for)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--progress", action="store_true", help="print a line after every stage of every step")
    ap.add_argument("--workload", default="mixed_k5", choices=["mixed_k5", "superquad_k8", "ellipsoids", "dielectric",
                                                            "dielectric_uq"],
                    help="mixed_k5: the k=5 icosphere ladder (default); superquad_k8: the superquadric ladder "
                         "|x|^4+|y|^4+|z|^4=1, k=8, to --max-level (s=6 does not fit both precisions' matrices "
                         "on one GPU); ellipsoids: 64 seeded ellipsoids x 16 "
                         "incidences, 3 levels each, Matern-3/2 covariance, all incidences solved together; "
                         "dielectric: the sphere experiment's rank-one DE second moment (PMCHWT, eps_r 2.1, k0 3) "
                         "on the icosphere ladder s=2..--max-level; dielectric_uq: the DE shape-uncertainty second "
                         "moment (radial Gaussian covariance 0.01, 0.5) on the same ladder")
    ap.add_argument("--shapes", type=int, default=64, help="ellipsoids: number of shapes")
    ap.add_argument("--workers", type=int, default=4,
                    help="ellipsoids: shapes in flight at once (fosb_second_moment_batch); 0 = one call per shape")
    ap.add_argument("--schedule", default="concurrent", choices=["concurrent", "sequential"],
                    help="concurrent: the library's two-stream pipeline (fosb_second_moment); sequential: the "
                         "step-by-step calls, timed per stage")
    ap.add_argument("--autotune", default="on", choices=["on", "off"],
                    help="GEMM tile autotuner (off: the built-in tile for every product)")
    ap.add_argument("--profile-mode", default="separate", choices=["separate", "timed"],
                    help="where the per-launch HIP events for the roofline are recorded: separate (one extra step "
                         "after the timed ones, same work) or timed (during the timed steps themselves)")
    ap.add_argument("--tune-load", default=None, metavar="JSON",
                    help="load a GEMM tile table ({bucket key: variant}, from --tune-dump) before the warmup")
    ap.add_argument("--tune-dump", default=None, metavar="JSON", help="write the GEMM tile table after the run")
    ap.add_argument("--reassemble", action="store_true",
                    help="mixed path: the finest level keeps no complex128 copy of Z (Zlow assembled in FP64 bands, "
                         "refinement residuals with Z re-assembled band by band); needed for superquad_k8 at s=6")
    ap.add_argument("--lowrank", action="store_true",
                    help="dielectric_uq: the low-rank covariance route (pivoted Cholesky to 1e-10) with shape-derivative "
                         "weights recomputed by source bands instead of stored")
    ap.add_argument("--lu-pivoting", type=int, default=0, choices=[0, 1],
                    help="mixed levels: 0 lets symmetric EFIE matrices skip pivoting, 1 always pivots")
    ap.add_argument("--no-stages", action="store_true",
                    help="skip the extra step through the step-by-step calls that times each stage")
    ap.add_argument("--save-var", default=None, metavar="NPZ",
                    help="write each path's variance of the last timed step to this .npz file")
    ap.add_argument("--certify", action="store_true",
                    help="after the timed steps, one untimed step per precision with opts.certify and refinement to "
                         "1e-13: backward error, 1-norm condition estimate and growth factor in the line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (HBM counter calibration)")
    ap.add_argument("--assembly-only", type=int, default=0, metavar="R",
                    help="only assemble the finest level of mixed_k5 (s = 5, k = 5) R times and print the times "
                         "(the assembly kernels' rate alone, for a kernel trace)")
    return ap.parse_args()


class Workload:
    def __init__(self, name: str, max_level: int):
        import workloads
        self.name = name
        self.w = workloads.workload(name, max_level=max_level)
        self.xh = self.w.angles

    def describe(self, npairs: int) -> str:
        w = self.w
        geo = "unit icosphere" if self.name == "mixed_k5" else "superquadric |x|^4+|y|^4+|z|^4=1"
        return (f"{self.name}: {geo} s={w.levels[0]}..{w.levels[-1]} (N up to {30 * 4 ** w.levels[-1]}), "
                f"k={w.k:g}, Gaussian radial cov ({w.sigma:g}, {w.ell:g}), L0={w.L0} L={w.L} ({npairs} pairs), "
                f"{w.n_angles} angles")


def gpu_setup(fosb, torch, ctx, W, reassemble=False):
    meshes = [fosb.Mesh(ctx, V, F) for V, F in W.w.meshes]
    Z = [None if (reassemble and i == len(meshes) - 1) else
         torch.empty((m.n_edges, m.n_edges), dtype=torch.complex128, device=ctx.torch_device)
         for i, m in enumerate(meshes)]
    return meshes, Z


PROGRESS = False


def _progress(msg):
    if PROGRESS:
        log(f"[bench]   {time.strftime('%H:%M:%S')} {msg}")


def one_step(fosb, torch, ctx, W, meshes, Z, Zlow, precision, cov, opts, stage_ev=None):
    w = W.w
    k = w.k
    L0, L = w.L0, w.L
    ev = stage_ev
    if ev:
        ev[0].record()
    for s, m, z in zip(w.levels, meshes, Z):
        if z is not None:
            fosb.assemble(ctx, m, k, opts, Z=z)
            _progress(f"assembled s={s}")
    if ev:
        ev[1].record()
    levels = []
    for s, m, z, zl in zip(w.levels, meshes, Z, Zlow):
        levels.append(fosb.Level(ctx, m, k, z, precision, w.dirs, w.pols, "radial", opts,
                                 Zlow=(zl if precision == fosb.MIXED else None)))
        _progress(f"factored s={s}")
    if ev:
        ev[2].record()
    st = fosb.Stats()
    blocks = fosb.correlation(ctx, levels, L0, L, cov, 0, stats=st)
    _progress("pairs solved")
    if ev:
        ev[3].record()
    var = fosb.far_field_moments(ctx, levels, L0, L, blocks, W.xh)
    _progress("far field")
    if ev:
        ev[4].record()
    return var, blocks, levels, st


def one_step_concurrent(fosb, ctx, W, meshes, Z, Zlow, precision, cov, opts, blocks):
    """The same pass through fosb_second_moment: finest level on the main
    stream, coarser levels and their pairs concurrently on the auxiliary one."""
    w = W.w
    st = fosb.Stats()
    var, _, _ = fosb.second_moment(ctx, meshes, w.L0, w.L, w.k, precision, cov, W.xh, w.dirs, w.pols, "radial", 0,
                                   Z=Z, Zlow=(Zlow if precision == fosb.MIXED else None), blocks=blocks,
                                   opts=opts, stats=st)
    _progress("pipeline done")
    return var, st


def algorithmic_flops(W):
    """8 flop per complex multiply-add: LU (8/3) N^3 per level, two-sided solve
    8 N1 N2 (N1 + N2) per pair, far-field contraction 24 n_a N1 N2 per pair."""
    from paper_2308_01457_amd import fosb
    N = {s: 30 * 4 ** s for s in W.w.levels}
    lu = sum(8.0 / 3.0 * n ** 3 for n in N.values())
    pairs = fosb.ct_pairs(W.w.L0, W.w.L)
    solve = sum(8.0 * N[a] * N[b] * (N[a] + N[b]) for a, b, _, _ in pairs)
    ff = sum(24.0 * W.w.n_angles * N[a] * N[b] for a, b, _, _ in pairs)
    return lu, solve, ff, len(pairs)


def assembly_point_pairs(W, n_gauss=5):
    """Point pairs the assembly integrates per step: 36 (6 x 6 points) per
    ordered non-touching triangle pair, and the Sauter-Schwab points of the
    touching ones (6, 5, 2 regions of n^4 points for identical, edge- and
    vertex-adjacent pairs)."""
    import scipy.sparse as sp
    reg = sing = 0
    for V, F in W.w.meshes:
        nt, nv = F.shape[0], V.shape[0]
        inc = sp.csr_matrix((np.ones(3 * nt), (np.repeat(np.arange(nt), 3), F.reshape(-1))), shape=(nt, nv))
        shared = (inc @ inc.T).tocoo()   # vertices shared by each ordered pair
        cnt = np.bincount(shared.data.astype(np.int64), minlength=4)
        touching = cnt[1] + cnt[2] + cnt[3]
        reg += 36 * (nt * nt - touching)
        sing += n_gauss ** 4 * (6 * cnt[3] + 5 * cnt[2] + 2 * cnt[1])
    return int(reg), int(sing)


def lu_flops_as_factored(levels):
    """Flops of the factorisations the levels kept: (8/3) N^3 for LU with
    partial pivoting, (4/3) N^3 for the symmetric factorisation (trailing
    updates of the lower triangle only)."""
    from paper_2308_01457_amd import fosb
    kinds = {lv.n: lv.factorization() for lv in levels}
    flop = sum((4.0 if k == fosb.FACTOR_SYM else 8.0) / 3.0 * n ** 3 for n, k in kinds.items())
    return flop, {str(n): ("symmetric" if k == fosb.FACTOR_SYM else "pivoted") for n, k in sorted(kinds.items())}


def stage_report(t, lu_f, solve_f, pname, sweeps, lu_kinds=None):
    """Seconds per stage of one step through the step-by-step calls, and each
    compute stage against its MFMA bound.  LU: the flops of the factorisations
    kept (lu_flops_as_factored) at the factor's precision.  Pairs: the two-sided solves, 8 N1 N2 (N1 + N2) per pair;
    on the mixed path each refinement sweep adds one FP64 residual product and
    one FP32 correction solve of the same flop count, so the stage executes
    (1 + sweeps) x that in FP32 and sweeps x that in FP64."""
    asm, lu, pairs, ff = t
    p32, p64 = PEAK["mixed"] * 1e12, PEAK["fp64"] * 1e12
    if pname == "mixed":
        f32, f64 = solve_f * (1 + sweeps), solve_f * sweeps
        lu_peak = p32
    else:
        f32, f64 = 0.0, solve_f
        lu_peak = p64
    bound = f32 / p32 + f64 / p64
    return {"assemble_s": asm, "far_field_s": ff,
            "lu_first_moment": {"seconds": lu, "algorithmic_flop": lu_f, "factorisation_by_n": lu_kinds,
                                "achieved_tflops": lu_f / lu / 1e12, "peak_tflops": lu_peak / 1e12,
                                "frac": lu_f / lu_peak / lu},
            "pairs": {"seconds": pairs, "algorithmic_flop": solve_f, "refinement_sweeps": sweeps,
                      "executed_flop_fp32": f32, "executed_flop_fp64": f64, "bound_seconds_at_peaks": bound,
                      "frac": bound / pairs}}


def run_gpu(args, W):
    import torch
    from paper_2308_01457_amd import fosb

    ctx = fosb.Context(0)
    fosb.autotune(ctx, 1 if args.autotune == "on" else 0)
    if args.tune_load:
        with open(args.tune_load) as f:
            fosb.autotune_load(ctx, {int(k): v for k, v in json.load(f).items()})
    cov = fosb.make_cov(W.w.cov_kind, W.w.sigma, W.w.ell)
    opts = fosb.opts_default(ir_tol=args.ir_tol, ir_max_sweeps=10, lu_pivoting=args.lu_pivoting)
    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    if args.reassemble and precs != ["mixed"]:
        raise SystemExit("--reassemble applies to the mixed path only (use --precision mixed)")
    meshes, Z = gpu_setup(fosb, torch, ctx, W, args.reassemble)
    Zlow = [None] * len(meshes)
    if "mixed" in precs:
        Zlow = [torch.empty((m.n_edges, m.n_edges), dtype=torch.complex64, device=ctx.torch_device) for m in meshes]
    lu_f, solve_f, ff_f, npairs = algorithmic_flops(W)
    out = {}
    blocks = [torch.empty((meshes[a - W.w.L0].n_edges, meshes[b - W.w.L0].n_edges), dtype=torch.complex128,
                          device=ctx.torch_device) for a, b, _, _ in fosb.ct_pairs(W.w.L0, W.w.L)]

    def step(prec, ev=None):
        if args.schedule == "concurrent":
            return one_step_concurrent(fosb, ctx, W, meshes, Z, Zlow, prec, cov, opts, blocks)
        var, blk, levels, st = one_step(fosb, torch, ctx, W, meshes, Z, Zlow, prec, cov, opts, ev)
        del blk, levels
        return var, st

    for pname in precs:
        prec = fosb.MIXED if pname == "mixed" else fosb.FP64
        log(f"[bench] {pname}: warmup {args.warmup}")
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        stage = np.zeros(4)
        times = []
        keep_var = None
        st = None
        prof_timed = not args.no_profile and args.profile_mode == "timed"
        if prof_timed:
            fosb.profile_enable(ctx, True)
        for i in range(args.steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)] if args.schedule == "sequential" else None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            var, st = step(prec, ev)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            times.append(dt)
            if ev:
                stage += [ev[j].elapsed_time(ev[j + 1]) * 1e-3 for j in range(4)]
            log(f"[bench] {pname} step {i}: {dt:.3f} s  (ir sweeps {st.ir_sweeps})")
            keep_var = var.cpu().numpy()
        t_step = float(np.mean(times))
        rec = {"seconds_per_step": t_step, "pair_solves_per_s": npairs / t_step, "ir_sweeps": int(st.ir_sweeps),
               "var": keep_var}
        if args.schedule == "sequential":
            stage /= max(1, args.steps)
            rec["stage_s"] = {"assemble": stage[0], "lu_first_moment": stage[1], "pairs": stage[2],
                              "far_field": stage[3]}
        if prof_timed:
            rec["profile"] = {k: (v[0] // max(1, args.steps), v[1] / max(1, args.steps), v[2] / max(1, args.steps),
                                  v[3] / max(1, args.steps)) for k, v in fosb.profile_read(ctx).items()}
            fosb.profile_enable(ctx, False)
        elif not args.no_profile:
            log(f"[bench] {pname}: profiled step")
            fosb.profile_enable(ctx, True)
            step(prec)
            prof = fosb.profile_read(ctx)
            fosb.profile_enable(ctx, False)
            rec["profile"] = prof
        if not args.no_stages and args.schedule == "concurrent":
            log(f"[bench] {pname}: staged step")
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            torch.cuda.synchronize()
            _, blk, lvs, sst = one_step(fosb, torch, ctx, W, meshes, Z, Zlow, prec, cov, opts, ev)
            torch.cuda.synchronize()
            lu_used, kinds = lu_flops_as_factored(lvs)
            del blk, lvs
            rec["stages"] = stage_report([ev[j].elapsed_time(ev[j + 1]) * 1e-3 for j in range(4)], lu_used,
                                         solve_f, pname, int(sst.ir_sweeps), kinds)
        if args.certify:
            log(f"[bench] {pname}: certified step")
            copts = fosb.opts_default(ir_tol=1e-13, ir_max_sweeps=20, certify=1, lu_pivoting=args.lu_pivoting)
            if args.schedule == "concurrent":
                _, cst = one_step_concurrent(fosb, ctx, W, meshes, Z, Zlow, prec, cov, copts, blocks)
            else:
                _, blk, lvs, cst = one_step(fosb, torch, ctx, W, meshes, Z, Zlow, prec, cov, copts)
                for lv in lvs:
                    kap, gro = lv.certificate()
                    cst.kappa1, cst.growth = max(cst.kappa1, kap), max(cst.growth, gro)
                del blk, lvs
            rec["certificate"] = {"ir_tol": 1e-13, "ir_sweeps": int(cst.ir_sweeps),
                                  "backward_error": cst.backward_error if prec == fosb.MIXED else None,
                                  "kappa1": cst.kappa1, "growth": cst.growth}
        out[pname] = rec
    if args.tune_dump:
        with open(args.tune_dump, "w") as f:
            json.dump({str(k): v for k, v in sorted(fosb.autotune_table(ctx).items())}, f, indent=0)
    return out, (lu_f, solve_f, ff_f, npairs)


def run_batched(args):
    """64 seeded ellipsoids (semi-axes U[0.7, 1.3], geodesic levels nu/4, nu/2,
    nu with nu ~ U{8..16}: 1280..5120 top triangles), k ~ U[1, 4], 16
    incidences each, Matern-3/2 radial covariance (0.01, ell ~ U[0.3, 0.8]),
    CT L0 = 0, L = 2 (3 pairs), 181 angles: 3 x 16 x 64 = 3072 level-pair
    solves per step, every shape through fosb_second_moment with its 16
    incidences stacked as right-hand sides."""
    import torch

    import workloads
    from paper_2308_01457_amd import fosb
    shapes = workloads.batched_ellipsoids(args.shapes, 16, 0)
    ctx = fosb.Context(0)
    fosb.autotune(ctx, 1 if args.autotune == "on" else 0)
    dev = ctx.torch_device
    xh = workloads.angles_xz(181)
    meshes = [[fosb.Mesh(ctx, V, F) for V, F in w.meshes] for w in shapes]
    N = [[m.n_edges for m in ms] for ms in meshes]
    pairs = fosb.ct_pairs(0, 2)
    opts = fosb.opts_default(ir_tol=args.ir_tol, ir_max_sweeps=10, lu_pivoting=args.lu_pivoting)
    npairs = len(pairs) * 16 * len(shapes)
    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    out = {}
    items = [{"meshes": ms, "L0": 0, "L": 2, "k": w.k, "dirs": w.dirs, "pols": w.pols,
              "cov": fosb.make_cov("matern32", w.sigma, w.ell)} for w, ms in zip(shapes, meshes)]
    if args.workers == 0:
        nmax = [max(n[i] for n in N) for i in range(3)]
        Zb = [torch.empty(nmax[i] ** 2, dtype=torch.complex128, device=dev) for i in range(3)]
        Zl = [torch.empty(nmax[i] ** 2, dtype=torch.complex64, device=dev) for i in range(3)]
        Bb = [torch.empty(nmax[a] * 16 * nmax[b], dtype=torch.complex128, device=dev) for a, b, _, _ in pairs]

    def step(prec):
        st = fosb.Stats()
        if args.workers > 0:
            return fosb.second_moment_batch(ctx, items, prec, xh, opts, args.workers, st), st
        res = []
        for it, n in zip(items, N):
            Z = [Zb[i][: n[i] ** 2].view(n[i], n[i]) for i in range(3)]
            Zlo = [Zl[i][: n[i] ** 2].view(n[i], n[i]) for i in range(3)] if prec == fosb.MIXED else None
            blocks = [Bb[p][: n[a] * 16 * n[b]].view(n[a], 16 * n[b]) for p, (a, b, _, _) in enumerate(pairs)]
            var, _, _ = fosb.second_moment(ctx, it["meshes"], 0, 2, it["k"], prec, it["cov"], xh, it["dirs"],
                                           it["pols"], "radial", -1, Z=Z, Zlow=Zlo, blocks=blocks, opts=opts,
                                           stats=st)
            res.append(var)
        return res, st

    for pname in precs:
        prec = fosb.MIXED if pname == "mixed" else fosb.FP64
        log(f"[bench] ellipsoids {pname}: warmup {args.warmup}")
        for _ in range(args.warmup):
            step(prec)
        times = []
        for i in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, st = step(prec)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            log(f"[bench] ellipsoids {pname} step {i}: {times[-1]:.3f} s  (ir sweeps {st.ir_sweeps})")
        t = float(np.mean(times))
        out[pname] = {"seconds_per_step": t, "pair_solves_per_s": npairs / t, "ir_sweeps": int(st.ir_sweeps),
                      "var": torch.stack([r.reshape(-1) for r in [x.reshape(-1) for x in res]]).cpu().numpy()}
        if not args.no_profile:
            log(f"[bench] ellipsoids {pname}: profiled step")
            fosb.profile_enable(ctx, True)
            step(prec)
            out[pname]["profile"] = fosb.profile_read(ctx)
            fosb.profile_enable(ctx, False)
    head = "mixed" if "mixed" in out else "fp64"
    line = {"metric": "Cor[u'] level-pair solves/sec + MFMA TFLOP/s, mixed vs FP64 at 1e-6 rel err",
            "value": out[head]["pair_solves_per_s"], "unit": "level-pair solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": out[head]["seconds_per_step"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "c64+f64" if head == "mixed" else "c128", "data": "synthetic",
            "config": {"workload": f"batched ellipsoids: {len(shapes)} shapes x 16 incidences, geodesic levels "
                                   f"nu/4, nu/2, nu (top 1280..5120 triangles), k ~ U[1,4], Matern-3/2 (0.01, "
                                   f"U[0.3,0.8]), L0=0 L=2 (3 pairs), 181 angles, incidences stacked",
                       "precision": head, "ir_tol": args.ir_tol, "level_pair_solves": npairs,
                       "shapes_in_flight": args.workers}}
    for pname, rec in out.items():
        line[pname] = {k: v for k, v in rec.items() if k not in ("var", "profile")}
    for pname, rec in out.items():   # dominant kernel of each path: its complex GEMM
        prof = rec.get("profile")
        if not prof:
            continue
        kname = "gemm_f32" if pname == "mixed" else "gemm_f64"
        n, sec, fl, by = prof[kname]
        ach = fl / sec / 1e12 if sec > 0 else 0.0
        key = "roofline" if pname == head else f"roofline_{pname}"
        line[key] = {"kernel": f"k_gemm<{'float' if pname == 'mixed' else 'double'}>", "bound": "mfma",
                     "achieved": ach, "peak": PEAK[pname], "unit": "TFLOP/s", "frac": ach / PEAK[pname],
                     "traffic": None, "launches": n, "avg_launch_us": sec / max(n, 1) * 1e6,
                     "algorithmic_flop_per_launch": fl / max(n, 1), "algorithmic_bytes_per_launch": by / max(n, 1),
                     "concurrent_streams": args.workers}
        line[f"kernel_profile_{pname}"] = {k: {"launches": v[0], "seconds": v[1],
                                               "tflops": (v[2] / v[1] / 1e12) if v[1] else 0,
                                               "gbs": (v[3] / v[1] / 1e9) if v[1] else 0} for k, v in prof.items()}
    if "mixed" in out and "fp64" in out:
        a, b = out["mixed"]["var"], out["fp64"]["var"]
        line["mixed_speedup_vs_fp64"] = out["fp64"]["seconds_per_step"] / out["mixed"]["seconds_per_step"]
        line["mixed_vs_fp64_var_rel_err"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(json.dumps(line), flush=True)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W):
    """The oracle on a bounded sample of the same workload, timed stage by stage
    on the host, then extrapolated to the full ladder:
    * levels s = 2, 3 (480 and 1920 RWG): assembly, LU + first moment, the
      (3,2) RHS correlation, two-sided solve and far-field contraction;
    * the oracle's LU routine (scipy.linalg.lu_factor, LAPACK getrf) on a
      seeded random complex matrix of the s = 4 size (7680): the LU stage
      dominates the full ladder, and this anchors its N^3 law at a size
      where the BLAS runs at its large-matrix rate.
    Cost laws: assembly ~ T^2 (from s = 3), LU ~ N^3 (from N = 7680), pair
    solve ~ N1 N2 (N1 + N2), RHS correlation and far field ~ N1 N2."""
    import scipy.linalg as sla

    import workloads
    from oracle import efie, mesh, uq
    blas = []
    try:
        from threadpoolctl import threadpool_info
        blas = [{k: p.get(k) for k in ("internal_api", "num_threads", "version")} for p in threadpool_info()]
    except Exception:
        pass
    cores = max([b.get("num_threads") or 1 for b in blas] + [1]) if blas else (os.cpu_count() or 1)
    w = W.w
    xh = W.xh
    t = {}
    lv = {}
    for s in (2, 3):
        V, F = workloads.icosphere(s)
        t0 = time.perf_counter()
        m = mesh.build(V, F)
        Z = efie.assemble(m, w.k)
        t[("asm", s)] = time.perf_counter() - t0
        t0 = time.perf_counter()
        lv[s] = uq.make_level(V, F, w.k, Z=Z)
        t[("lu", s)] = time.perf_counter() - t0
    t0 = time.perf_counter()
    C = uq.rhs_correlation(lv[3], lv[2], w.cov_kind, w.sigma, w.ell)
    t_c = time.perf_counter() - t0
    t0 = time.perf_counter()
    S = uq.two_sided_solve(lv[3], lv[2], C)
    t_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    FF3 = uq.far_field_matrix(lv[3], xh)
    FF2 = uq.far_field_matrix(lv[2], xh)
    uq.pair_variance(FF3, S, FF2)
    t_f = time.perf_counter() - t0
    n4 = 30 * 4 ** 4
    rng = np.random.Generator(np.random.PCG64(4))
    A = rng.standard_normal((n4, n4)) + 1j * rng.standard_normal((n4, n4))
    t0 = time.perf_counter()
    sla.lu_factor(A, overwrite_a=True, check_finite=False)
    t_lu4 = time.perf_counter() - t0
    del A
    sample_s = sum(t.values()) + t_c + t_s + t_f + t_lu4
    N = {s: 30 * 4 ** s for s in w.levels}
    T = {s: 20 * 4 ** s for s in w.levels}
    proj = 0.0
    for s in w.levels:
        proj += t[("asm", 3)] * (T[s] / T[3]) ** 2 + t_lu4 * (N[s] / n4) ** 3
    from paper_2308_01457_amd import fosb
    pairs = fosb.ct_pairs(w.L0, w.L)
    base_s = 8.0 * N[3] * N[2] * (N[3] + N[2])
    for a, b, _, _ in pairs:
        proj += t_s * 8.0 * N[a] * N[b] * (N[a] + N[b]) / base_s
        proj += (t_c + t_f) * N[a] * N[b] / (N[3] * N[2])
    return {"value": len(pairs) / proj, "unit": "level-pair solves/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(), "blas": blas,
            "sample": (f"oracle (numpy/scipy FP64) timed on levels s=2,3 of the ladder (assembly, LU + first moment, "
                       f"the (3,2) RHS correlation, two-sided solve and far-field contraction) and its LU routine "
                       f"on a random complex {n4} x {n4} matrix ({t_lu4:.1f} s, {8.0 / 3.0 * n4 ** 3 / t_lu4 / 1e9:.0f}"
                       f" GFLOP/s); {sample_s:.1f} s in all; extrapolated to s=2..5 by T^2 (assembly, from s=3), "
                       f"N^3 (LU, from N={n4}), N1 N2 (N1+N2) (pair solve); projected {proj:.0f} s per step"),
            "projected_seconds_per_step": proj,
            "stage_seconds_sample": {"assembly_s3": t[("asm", 3)], "lu_first_moment_s3": t[("lu", 3)],
                                     "lu_n7680": t_lu4, "rhs_correlation_32": t_c, "two_sided_32": t_s,
                                     "far_field_32": t_f}}


def calibrate_copy():
    """Plain device-to-device copy of a known size: the reference that scales
    rocprofv3's FETCH_SIZE / WRITE_SIZE counters to HBM bytes."""
    import torch
    n = 1 << 28                                     # 2^28 float32 = 1 GiB
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                      "launches": 5}), flush=True)


def assembly_only(reps):
    """The finest level's EFIE assembly of mixed_k5 (unit icosphere s = 5,
    N = 30720, k = 5), `reps` times on one context: the assembly kernels' rate
    with nothing else on the chip."""
    import torch

    import workloads
    from paper_2308_01457_amd import fosb
    w = workloads.workload("mixed_k5")
    ctx = fosb.Context(0)
    mesh = fosb.Mesh(ctx, *w.meshes[-1])
    Z = torch.empty((mesh.n_edges, mesh.n_edges), dtype=torch.complex128, device=ctx.torch_device)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fosb.assemble(ctx, mesh, w.k, Z=Z)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    print(json.dumps({"assembly": "mixed_k5 s=5", "n_edges": mesh.n_edges, "k": w.k, "seconds": times}), flush=True)


def run_dielectric(args):
    """The sphere experiment's DE second moment: unit icosphere s = 2..L
    (2N up to 2 x 30 x 4^L), eps_r 2.1, mu_r 1, k0 3, incidence d = e_x,
    p = e_z, rank-one right-hand side M2[f] = f (x) f over the CT index set
    (L0 = 2), far-field second moment at 1801 angles in the plane z = 0.  A step
    assembles every PMCHWT matrix, factors each level and solves its first
    moment, forms and solves every CT pair and contracts the far field.
    dielectric_uq: the same ladder with the shape-uncertainty second moment
    (radial Gaussian amplitude, sigma 0.01, ell 0.5): each level also builds
    its shape-derivative weights, and each pair's right-hand side is
    W_l1 K W_l2^H."""
    import torch

    import workloads
    from paper_2308_01457_amd import fosb
    K0, EPS, MU, L0 = 3.0, 2.1, 1.0, 2
    L = args.max_level
    D, P = (1.0, 0.0, 0.0), (0.0, 0.0, 1.0)
    xh = workloads.angles_xy(1801)
    ctx = fosb.Context(0)
    meshes = [fosb.Mesh(ctx, *workloads.icosphere(s)) for s in range(L0, L + 1)]
    pairs = fosb.ct_pairs(L0, L)
    npairs = len(pairs)
    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    Z = [torch.empty((2 * m.n_edges, 2 * m.n_edges), dtype=torch.complex128, device=ctx.torch_device)
         for m in meshes]
    Zlow = [torch.empty((2 * m.n_edges, 2 * m.n_edges), dtype=torch.complex64, device=ctx.torch_device)
            for m in meshes] if "mixed" in precs else [None] * len(meshes)
    blocks = [torch.empty((2 * meshes[a - L0].n_edges, 2 * meshes[b - L0].n_edges), dtype=torch.complex128,
                          device=ctx.torch_device) for a, b, _, _ in pairs] if not args.lowrank else None
    opts = fosb.opts_default(ir_tol=args.ir_tol, ir_max_sweeps=10, lu_pivoting=args.lu_pivoting)
    uq = args.workload == "dielectric_uq"
    cov = fosb.make_cov("gaussian", 0.01, 0.5) if uq else None

    def step(prec):
        levels = []
        for m, z, zl in zip(meshes, Z, Zlow):
            fosb.assemble_pmchwt(ctx, m, K0, EPS, MU, opts, Z=z)
            levels.append(fosb.Level.pmchwt(ctx, m, K0, EPS, MU, z, prec, dirs=[D], pols=[P], opts=opts,
                                            Zlow=zl if prec == fosb.MIXED else None,
                                            field="radial" if uq else None, streamed=uq and args.lowrank))
        st = fosb.Stats()
        if uq and args.lowrank:
            lr = fosb.LowRank(ctx, levels, cov, 8192, 1e-10)
            var = lr.far_field_moments(L0, L, xh, stats=st)
            step.rank = lr.rank
            lr.close()
        else:
            fosb.correlation(ctx, levels, L0, L, cov, 0, blocks=blocks, stats=st)
            var = fosb.far_field_moments(ctx, levels, L0, L, blocks, xh)
        for lv in levels:
            lv.close()
        return var, st

    out = {}
    for pname in precs:
        prec = fosb.MIXED if pname == "mixed" else fosb.FP64
        log(f"[bench] dielectric {pname}: warmup {args.warmup}")
        for _ in range(args.warmup):
            step(prec)
        times = []
        for i in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            var, st = step(prec)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            log(f"[bench] dielectric {pname} step {i}: {times[-1]:.3f} s  (ir sweeps {st.ir_sweeps})")
        t = float(np.mean(times))
        out[pname] = {"seconds_per_step": t, "pair_solves_per_s": npairs / t, "ir_sweeps": int(st.ir_sweeps),
                      "var": var.cpu().numpy()}
        if not args.no_profile:
            log(f"[bench] dielectric {pname}: profiled step")
            fosb.profile_enable(ctx, True)
            step(prec)
            out[pname]["profile"] = fosb.profile_read(ctx)
            fosb.profile_enable(ctx, False)
    head = "mixed" if "mixed" in out else "fp64"
    n_top = 2 * meshes[-1].n_edges
    line = {"metric": "Cor[u'] level-pair solves/sec + MFMA TFLOP/s, mixed vs FP64 at 1e-6 rel err",
            "value": out[head]["pair_solves_per_s"], "unit": "level-pair solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": out[head]["seconds_per_step"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "c64+f64" if head == "mixed" else "c128", "data": "synthetic",
            "config": {"workload": (f"dielectric sphere: unit icosphere s={L0}..{L} (PMCHWT, 2N up to {n_top}), "
                                    f"eps_r 2.1, mu_r 1, k0 3, d = e_x, p = e_z, "
                                    + ("shape-uncertainty second moment, radial Gaussian amplitude (0.01, 0.5)"
                                       if uq else "rank-one RHS f (x) f (sphere experiment)")
                                    + f", L0={L0} L={L} ({npairs} pairs), 1801 angles in z = 0"),
                       "precision": head, "ir_tol": args.ir_tol,
                       "route": "low-rank covariance (tol 1e-10), streamed weights" if (uq and args.lowrank) else
                                ("dense covariance" if uq else "rank-one")}}
    if uq and args.lowrank:
        line["config"]["lowrank_rank"] = getattr(step, "rank", None)
    for pname, rec in out.items():
        line[pname] = {k: v for k, v in rec.items() if k not in ("var", "profile")}
    with open(os.path.join(ROOT, "tests", "golden", "dielectric_mie_k3.json")) as f:
        mie_f2 = np.asarray(json.load(f)["abs_F2"])   # |F_c|^2 of the Mie series, stored
    for pname, rec in out.items():   # discretisation + CT error against the mesh-free value
        if uq:
            break
        line[pname]["abs_F2_vs_mie_rel_err"] = float(np.linalg.norm(rec["var"] - mie_f2) / np.linalg.norm(mie_f2))
        line[pname]["abs_Fz2_vs_mie_rel_err"] = float(np.linalg.norm(rec["var"][2] - mie_f2[2]) /
                                                      np.linalg.norm(mie_f2[2]))
    if "mixed" in out and "fp64" in out:
        a, b = out["mixed"]["var"], out["fp64"]["var"]
        line["mixed_speedup_vs_fp64"] = out["fp64"]["seconds_per_step"] / out["mixed"]["seconds_per_step"]
        line["mixed_vs_fp64_var_rel_err"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    for pname, rec in out.items():
        prof = rec.get("profile")
        if not prof:
            continue
        line[f"kernel_profile_{pname}"] = {k: {"launches": v[0], "seconds": v[1],
                                               "tflops": (v[2] / v[1] / 1e12) if v[1] else 0,
                                               "gbs": (v[3] / v[1] / 1e9) if v[1] else 0} for k, v in prof.items()}
        kname = "gemm_f32" if pname == "mixed" else "gemm_f64"
        n, sec, fl, by = prof[kname]
        ach = fl / sec / 1e12 if sec > 0 else 0.0
        key = "roofline" if pname == head else f"roofline_{pname}"
        line[key] = {"kernel": f"k_gemm<{'float' if pname == 'mixed' else 'double'}>", "bound": "mfma",
                     "achieved": ach, "peak": PEAK[pname], "unit": "TFLOP/s", "frac": ach / PEAK[pname],
                     "traffic": None, "launches": n, "avg_launch_us": sec / max(n, 1) * 1e6,
                     "algorithmic_flop_per_launch": fl / max(n, 1), "algorithmic_bytes_per_launch": by / max(n, 1)}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    global PROGRESS
    PROGRESS = args.progress
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.assembly_only > 0:
        assembly_only(args.assembly_only)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "ellipsoids":
        run_batched(args)
        return
    if args.workload in ("dielectric", "dielectric_uq"):
        run_dielectric(args)
        return
    W = Workload(args.workload, args.max_level)
    gpu, (lu_f, solve_f, ff_f, npairs) = run_gpu(args, W)
    head = "mixed" if "mixed" in gpu else "fp64"
    h = gpu[head]
    line = {
        "metric": "Cor[u'] level-pair solves/sec + MFMA TFLOP/s, mixed vs FP64 at 1e-6 rel err",
        "value": h["pair_solves_per_s"],
        "unit": "level-pair solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["seconds_per_step"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64" if head == "mixed" else "c128",
        "data": "synthetic",
        "config": {"workload": W.describe(npairs),
                   "precision": head, "schedule": args.schedule, "ir_tol": args.ir_tol, "autotune": args.autotune,
                   "finest_level_reassembled": bool(args.reassemble), "lu_pivoting": args.lu_pivoting,
                   "profile_mode": args.profile_mode},
        "algorithmic_flop_per_step": {"lu": lu_f, "pair_solves": solve_f, "far_field": ff_f},
    }
    for pname, rec in gpu.items():
        line[pname] = {k: v for k, v in rec.items() if k not in ("var", "profile")}
    if args.save_var:
        np.savez(args.save_var, **{p: r["var"] for p, r in gpu.items()})
    mie_file = os.path.join(ROOT, "tests", "golden", "mie_shape_oracle.json")
    if W.name == "mixed_k5" and W.w.levels[-1] == 5 and os.path.exists(mie_file):
        with open(mie_file) as f:
            mie = np.asarray(json.load(f)["variance"]["5.0"])
        for pname, rec in gpu.items():   # discretisation + CT error against the mesh-free value
            line[pname]["vs_mie_shape_rel_err"] = float(np.linalg.norm(rec["var"] - mie) / np.linalg.norm(mie))
    if "mixed" in gpu and "fp64" in gpu:
        v64, v32 = gpu["fp64"]["var"], gpu["mixed"]["var"]
        line["mixed_speedup_vs_fp64"] = gpu["fp64"]["seconds_per_step"] / gpu["mixed"]["seconds_per_step"]
        line["mixed_vs_fp64_var_rel_err"] = float(np.linalg.norm(v32 - v64) / np.linalg.norm(v64))
    prof = h.get("profile")
    if prof:
        kname = "gemm_f32" if head == "mixed" else "gemm_f64"
        n, sec, fl, by = prof[kname]
        ach = fl / sec / 1e12 if sec > 0 else 0.0
        line["roofline"] = {"kernel": f"k_gemm<{'float' if head == 'mixed' else 'double'}>", "bound": "mfma",
                            "achieved": ach, "peak": PEAK[head], "unit": "TFLOP/s", "frac": ach / PEAK[head],
                            "traffic": measured_traffic() if head == "mixed" else None,
                            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                            "copy-calibrated)",
                            "launches": n, "avg_launch_us": sec / max(n, 1) * 1e6,
                            "algorithmic_flop_per_launch": fl / max(n, 1),
                            "algorithmic_bytes_per_launch": by / max(n, 1)}
        line["kernel_profile"] = {k: {"launches": v[0], "seconds": v[1], "tflops": (v[2] / v[1] / 1e12) if v[1] else 0,
                                      "gbs": (v[3] / v[1] / 1e9) if v[1] else 0} for k, v in prof.items()}
        reg, sing = assembly_point_pairs(W)
        asec = prof["assemble"][1]
        line["assembly"] = {"regular_point_pairs": reg, "singular_point_pairs": sing, "seconds": asec,
                            "point_pairs_per_s": (reg + sing) / asec if asec > 0 else None,
                            "note": "all assembly kernels of one step (regular, touching, gather), FP64"}
    prof64 = gpu.get("fp64", {}).get("profile") if head == "mixed" else None
    if prof64:   # the FP64 path's dominant kernel, for the mixed-versus-FP64 comparison
        n, sec, fl, by = prof64["gemm_f64"]
        ach = fl / sec / 1e12 if sec > 0 else 0.0
        line["roofline_fp64"] = {"kernel": "k_gemm<double>", "bound": "mfma", "achieved": ach, "peak": PEAK["fp64"],
                                 "unit": "TFLOP/s", "frac": ach / PEAK["fp64"], "traffic": None,
                                 "launches": n, "avg_launch_us": sec / max(n, 1) * 1e6,
                                 "algorithmic_flop_per_launch": fl / max(n, 1),
                                 "algorithmic_bytes_per_launch": by / max(n, 1)}
        line["kernel_profile_fp64"] = {k: {"launches": v[0], "seconds": v[1],
                                           "tflops": (v[2] / v[1] / 1e12) if v[1] else 0,
                                           "gbs": (v[3] / v[1] / 1e9) if v[1] else 0} for k, v in prof64.items()}
    if not args.no_cpu_baseline and W.name == "mixed_k5":
        log("[bench] cpu baseline (oracle sample)")
        line["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
