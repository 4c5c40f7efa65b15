"""fosb_second_moment (two-stream schedule of the whole hot path) against the
step-by-step calls and the oracle, on the plain FP64 workload (unit icosphere
s=1..3, k=1, L0=1, L=3, 181 angles, radial Gaussian covariance 0.01 / 0.5).

The kernels are deterministic and the schedule only changes which stream
runs them, so blocks and variance must equal the step-by-step results
exactly."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K1 = 1.0
SIG, ELL = 0.01, 0.5


@pytest.fixture(scope="module")
def fz():
    import torch
    from paper_2308_01457_amd import fosb
    assert torch.cuda.is_available()
    return fosb, fosb.Context(0), torch


def _step_by_step(fosb, ctx, meshes, L0, L, prec, cov, xh, opts=None):
    levels = []
    for m in meshes:
        Z = fosb.assemble(ctx, m, K1, opts)
        levels.append(fosb.Level(ctx, m, K1, Z, prec, opts=opts))
    blocks = fosb.correlation(ctx, levels, L0, L, cov)
    var = fosb.far_field_moments(ctx, levels, L0, L, blocks, xh)
    return var.cpu().numpy(), [b.cpu().numpy() for b in blocks], levels


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pipeline_equals_step_by_step(fz, oracle_levels, precision):
    fosb, ctx, torch = fz
    from oracle import uq
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    xh = workloads.angles_xz(181)
    cov = fosb.make_cov("gaussian", SIG, ELL)
    meshes = [fosb.Mesh(ctx, *workloads.icosphere(s)) for s in (1, 2, 3)]
    print(f"[gpu] pipeline {precision} s=1..3", flush=True)
    st = fosb.Stats()
    var, blocks, _ = fosb.second_moment(ctx, meshes, 1, 3, K1, prec, cov, xh, stats=st)
    v_ref, b_ref, _ = _step_by_step(fosb, ctx, meshes, 1, 3, prec, cov, xh)
    assert np.array_equal(var.cpu().numpy(), v_ref)
    for b, r in zip(blocks, b_ref):
        assert np.array_equal(b.cpu().numpy(), r)
    olv = {s: oracle_levels(s) for s in (1, 2, 3)}
    Vo = uq.second_moment(None, K1, 1, 3, "gaussian", SIG, ELL, xh, levels=olv)[0]
    e = float(np.linalg.norm(var.cpu().numpy() - Vo) / np.linalg.norm(Vo))
    print(f"[gpu]   variance vs oracle {e:.2e}, sweeps {st.ir_sweeps}, solves {st.n_solves}", flush=True)
    assert e < (1e-10 if precision == "fp64" else 1e-5)
    assert st.n_solves == 3


def test_pipeline_equals_step_by_step_symmetric_top(fz):
    """The same exact equality, mixed precision, with the finest level (s = 4,
    N = 7680, k = 5) in the symmetric FP32 factorisation: the pass takes that
    level's complex64 copy from the assembly's gather, the step-by-step calls
    convert the assembled matrix, and the two copies must agree bit for bit."""
    fosb, ctx, torch = fz
    k = 5.0
    xh = workloads.angles_xz(61)
    cov = fosb.make_cov("gaussian", SIG, ELL)
    meshes = [fosb.Mesh(ctx, *workloads.icosphere(s)) for s in (2, 3, 4)]
    print("[gpu] pipeline mixed s=2..4, k=5 (symmetric top level)", flush=True)
    var, blocks, lv = fosb.second_moment(ctx, meshes, 2, 4, k, fosb.MIXED, cov, xh, keep_levels=True)
    ref = []
    for m in meshes:
        Z = fosb.assemble(ctx, m, k)
        ref.append(fosb.Level(ctx, m, k, Z, fosb.MIXED))
    assert lv[-1].factorization() == fosb.FACTOR_SYM and ref[-1].factorization() == fosb.FACTOR_SYM
    for a, b in zip(lv, ref):
        assert torch.equal(a.first_moment(0), b.first_moment(0))
    b_ref = fosb.correlation(ctx, ref, 2, 4, cov)
    v_ref = fosb.far_field_moments(ctx, ref, 2, 4, b_ref, xh)
    assert torch.equal(var, v_ref)
    for b, r in zip(blocks, b_ref):
        assert torch.equal(b, r)


def test_pipeline_single_level_and_handles(fz):
    """L0 = L (no auxiliary work), and the returned handles serve the adjoint."""
    fosb, ctx, torch = fz
    xh = workloads.angles_xz(37)
    cov = fosb.make_cov("gaussian", SIG, ELL)
    meshes = [fosb.Mesh(ctx, *workloads.icosphere(2))]
    print("[gpu] pipeline single level s=2", flush=True)
    var, blocks, levels = fosb.second_moment(ctx, meshes, 2, 2, K1, fosb.FP64, cov, xh, keep_levels=True)
    v_ref, b_ref, lv_ref = _step_by_step(fosb, ctx, meshes, 2, 2, fosb.FP64, cov, xh)
    assert np.array_equal(var.cpu().numpy(), v_ref)
    ones = torch.ones((3, 37), dtype=torch.float64, device=ctx.torch_device)
    g1 = fosb.far_field_moments_backward(ctx, levels, 2, 2, cov, xh, ones).cpu().numpy()
    g2 = fosb.far_field_moments_backward(ctx, lv_ref, 2, 2, cov, xh, ones).cpu().numpy()
    assert np.array_equal(g1, g2)
    print("[gpu] pipeline with handles kept, s=1..3 mixed", flush=True)
    meshes = [fosb.Mesh(ctx, *workloads.icosphere(s)) for s in (1, 2, 3)]
    var, blocks, levels = fosb.second_moment(ctx, meshes, 1, 3, K1, fosb.MIXED, cov, xh, keep_levels=True)
    g3 = fosb.far_field_moments_backward(ctx, levels, 1, 3, cov, xh, ones).cpu().numpy()
    assert abs(g3[2] - float(var.sum().item())) < 1e-10 * abs(g3[2])


def test_pipeline_rejects_bad_ladders(fz):
    fosb, ctx, torch = fz
    xh = workloads.angles_xz(5)
    cov = fosb.make_cov("gaussian", SIG, ELL)
    m1, m2 = (fosb.Mesh(ctx, *workloads.icosphere(s)) for s in (1, 2))
    with pytest.raises(fosb.FosbError) as e:
        fosb.second_moment(ctx, [m2, m1], 1, 2, K1, fosb.FP64, cov, xh)     # fine to coarse
    assert e.value.name == "E_INVALID"
    Z = [torch.empty((m.n_edges, m.n_edges), dtype=torch.complex128, device=ctx.torch_device) for m in (m1, m2)]
    blocks = [torch.empty((1, 1), dtype=torch.complex128, device=ctx.torch_device) for _ in range(3)]
    with pytest.raises(fosb.FosbError) as e:                                # n_levels != L - L0 + 1
        fosb.second_moment(ctx, [m1, m2], 1, 3, K1, fosb.FP64, cov, xh, Z=Z, blocks=blocks)
    assert e.value.name == "E_INVALID"
    with pytest.raises(fosb.FosbError) as e:
        fosb.second_moment(ctx, [m1, m2], 1, 2, -1.0, fosb.FP64, cov, xh)   # wavenumber
    assert e.value.name == "E_INVALID"


def test_stacked_incidences_ellipsoid_vs_oracle(fz):
    """dir = -1: three random incidences solved together on a geodesic
    ellipsoid ladder (nu = 2, 4, 8: 80 / 320 / 1280 triangles), Matern-3/2
    covariance, against the oracle run once per incidence (FP64 1e-10) and
    against the single-incidence pipeline (mixed)."""
    fosb, ctx, torch = fz
    from oracle import uq
    shape = workloads.batched_ellipsoids(n_shapes=1, n_dirs=3, seed=4)[0]
    axes = tuple(shape.extra["axes"])
    ladder = [workloads.ellipsoid(nu, axes) for nu in (2, 4, 8)]
    k, ell = shape.k, shape.ell
    xh = workloads.angles_xz(61)
    cov = fosb.make_cov("matern32", 0.01, ell)
    meshes = [fosb.Mesh(ctx, V, F) for V, F in ladder]
    print(f"[gpu] stacked incidences: ellipsoid axes {np.round(axes, 3)}, k={k:.3f}, ell={ell:.3f}", flush=True)
    var, blocks, _ = fosb.second_moment(ctx, meshes, 0, 2, k, fosb.FP64, cov, xh, shape.dirs, shape.pols, dir=-1)
    var = var.cpu().numpy()
    Zs = {}
    for d in range(3):
        olv = {}
        for s, (V, F) in enumerate(ladder):
            olv[s] = uq.make_level(V, F, k, shape.dirs[d], shape.pols[d], Z=Zs.get(s))
            Zs[s] = olv[s].Z
        Vo = uq.second_moment(None, k, 0, 2, "matern32", 0.01, ell, xh, levels=olv)[0]
        e = float(np.linalg.norm(var[d] - Vo) / np.linalg.norm(Vo))
        print(f"[gpu]   incidence {d}: variance vs oracle {e:.2e}", flush=True)
        assert e < 1e-10
    vm, _, _ = fosb.second_moment(ctx, meshes, 0, 2, k, fosb.MIXED, cov, xh, shape.dirs, shape.pols, dir=-1)
    for d in range(3):
        v1, _, _ = fosb.second_moment(ctx, meshes, 0, 2, k, fosb.MIXED, cov, xh, shape.dirs, shape.pols, dir=d)
        e = float(np.linalg.norm(vm[d].cpu().numpy() - v1.cpu().numpy()) / np.linalg.norm(v1.cpu().numpy()))
        print(f"[gpu]   mixed stacked vs single incidence {d}: {e:.2e}", flush=True)
        assert e < 1e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_per_shape(fz, precision):
    """fosb_second_moment_batch over three ellipsoid ladders of uneven sizes
    (two workers) equals fosb_second_moment(dir = -1) shape by shape."""
    fosb, ctx, torch = fz
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    xh = workloads.angles_xz(31)
    shapes = workloads.batched_ellipsoids(n_shapes=3, n_dirs=2, seed=11)
    items = []
    for w, nus in zip(shapes, ((1, 2, 4), (2, 4, 6), (1, 3, 5))):
        ms = [fosb.Mesh(ctx, *workloads.ellipsoid(nu, tuple(w.extra["axes"]))) for nu in nus]
        items.append({"meshes": ms, "L0": 0, "L": 2, "k": w.k, "dirs": w.dirs, "pols": w.pols,
                      "cov": fosb.make_cov("matern32", w.sigma, w.ell)})
    print(f"[gpu] batch of 3 shapes, 2 workers, {precision}", flush=True)
    st = fosb.Stats()
    out = fosb.second_moment_batch(ctx, items, prec, xh, n_workers=2, stats=st)
    assert st.n_solves == 3 * 3 * 2
    for it, v in zip(items, out):
        ref, _, _ = fosb.second_moment(ctx, it["meshes"], 0, 2, it["k"], prec, it["cov"], xh, it["dirs"],
                                       it["pols"], dir=-1)
        assert np.array_equal(v.cpu().numpy(), ref.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_does_not_change_results(fz, precision):
    """GEMM tile shapes differ only in how work is spread: with the autotuner
    off (built-in shape) and on (fresh table, every size bucket timed) the
    whole pass gives identical bits."""
    fosb, ctx, torch = fz
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    xh = workloads.angles_xz(31)
    cov = fosb.make_cov("gaussian", SIG, ELL)
    meshes = [fosb.Mesh(ctx, *workloads.icosphere(s)) for s in (1, 2, 3)]
    try:
        fosb.autotune(ctx, 0)
        v0, b0, _ = fosb.second_moment(ctx, meshes, 1, 3, K1, prec, cov, xh)
        fosb.autotune(ctx, 2)
        v1, b1, _ = fosb.second_moment(ctx, meshes, 1, 3, K1, prec, cov, xh)
        n = fosb.autotune(ctx, -1)
    finally:
        fosb.autotune(ctx, 1)
    print(f"[gpu] autotune {precision}: {n} tuned buckets", flush=True)
    assert n > 0
    assert np.array_equal(v0.cpu().numpy(), v1.cpu().numpy())
    for x, y in zip(b0, b1):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())


def test_autotune_table_export_and_load(fz):
    """A tuned table exported from one context and loaded into a fresh one
    settles the same buckets (no timing) and gives identical results; a
    variant out of range is rejected and loads nothing."""
    fosb, ctx, torch = fz
    xh = workloads.angles_xz(31)
    cov = fosb.make_cov("gaussian", SIG, ELL)
    c1, c2 = fosb.Context(0), fosb.Context(0)
    fosb.autotune(c1, 2)
    m1 = [fosb.Mesh(c1, *workloads.icosphere(s)) for s in (1, 2, 3)]
    v1, _, _ = fosb.second_moment(c1, m1, 1, 3, K1, fosb.MIXED, cov, xh)
    table = fosb.autotune_table(c1)
    print(f"[gpu] autotune table: {len(table)} buckets", flush=True)
    assert len(table) == fosb.autotune(c1, -1) > 0
    fosb.autotune(c2, 2)
    fosb.autotune_load(c2, table)
    assert fosb.autotune_table(c2) == table
    m2 = [fosb.Mesh(c2, *workloads.icosphere(s)) for s in (1, 2, 3)]
    v2, _, _ = fosb.second_moment(c2, m2, 1, 3, K1, fosb.MIXED, cov, xh)
    assert fosb.autotune_table(c2) == table          # every bucket was already settled
    assert np.array_equal(v1.cpu().numpy(), v2.cpu().numpy())
    key = next(iter(table))
    with pytest.raises(fosb.FosbError) as e:
        fosb.autotune_load(c2, {key + 1: 0, key: 7})
    assert e.value.name == "E_INVALID"
    assert fosb.autotune_table(c2) == table


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_batch_against_oracle_golden(fz, precision, tol):
    """Batched workload at full size: shapes 1 (geodesic frequency 16, N up to
    7680) and 2 (frequency 8) of the 64-ellipsoid batch (seed 0), each with
    its 16 incidences, Matern-3/2 covariance and 181 angles, through
    fosb_second_moment_batch (two workers, incidences stacked), against
    tests/golden/ellipsoids_oracle.json written by make_ellipsoids_golden.py
    from the oracle alone (one incidence at a time).  Per incidence: relative
    2-norm of the variance over (component, angle); the mixed path refines to
    the benchmark's 1e-7."""
    fosb, ctx, torch = fz
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ellipsoids_oracle.json")) as f:
        gold = json.load(f)
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    batch = workloads.batched_ellipsoids(64, 16, seed=0)
    xh = workloads.angles_xz(181)
    items = []
    for rec in gold["shapes"]:
        w = batch[rec["index"]]
        assert [int(x) for x in w.extra["nu"]] == rec["nu"] and abs(w.k - rec["k"]) < 1e-15
        ms = [fosb.Mesh(ctx, V, F) for V, F in w.meshes]
        items.append({"meshes": ms, "L0": 0, "L": 2, "k": w.k, "dirs": w.dirs, "pols": w.pols,
                      "cov": fosb.make_cov("matern32", w.sigma, w.ell)})
    print(f"[gpu] batch golden {precision}: shapes {[r['index'] for r in gold['shapes']]}", flush=True)
    opts = fosb.opts_default(ir_tol=1e-7) if prec == fosb.MIXED else None
    out = fosb.second_moment_batch(ctx, items, prec, xh, opts=opts, n_workers=2)
    for rec, v in zip(gold["shapes"], out):
        v = v.cpu().numpy()
        ref = np.asarray(rec["variance"])
        errs = [float(np.linalg.norm(v[d] - ref[d]) / np.linalg.norm(ref[d])) for d in range(ref.shape[0])]
        print(f"[gpu]   shape {rec['index']}: worst incidence {max(errs):.2e}", flush=True)
        assert max(errs) < tol
