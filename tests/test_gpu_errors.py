"""Error paths of the C ABI on a GPU context: every documented status is
returned as an error (never a crash), with the context still usable after.

* E_SINGULAR: factorising an all-zero matrix (exactly zero first pivot).
* E_NOCONV: mixed refinement capped at one sweep with an unreachable tolerance.
* E_WORKSPACE / E_INVALID: short leading dimensions, foreign handles, bad
  incidence index, bad covariance, bad context device."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fz():
    import torch
    from paper_2308_01457_amd import fosb
    assert torch.cuda.is_available()
    return fosb, fosb.Context(0), torch


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_matrix_is_singular(fz, precision):
    fosb, ctx, torch = fz
    m = fosb.Mesh(ctx, *workloads.icosphere(1))
    Z = torch.zeros((m.n_edges, m.n_edges), dtype=torch.complex128, device=ctx.torch_device)
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    print(f"[gpu] singular matrix {precision}", flush=True)
    with pytest.raises(fosb.FosbError) as e:
        fosb.Level(ctx, m, 1.0, Z, prec)
    assert e.value.name == "E_SINGULAR"
    # the context still works
    Z = fosb.assemble(ctx, m, 1.0)
    lv = fosb.Level(ctx, m, 1.0, Z, prec)
    assert torch.isfinite(lv.first_moment().abs()).all()


def test_refinement_not_converged(fz):
    fosb, ctx, torch = fz
    m = fosb.Mesh(ctx, *workloads.icosphere(2))
    Z = fosb.assemble(ctx, m, 1.0)
    print("[gpu] refinement capped at one sweep, tolerance 1e-300", flush=True)
    with pytest.raises(fosb.FosbError) as e:
        fosb.Level(ctx, m, 1.0, Z, fosb.MIXED, opts=fosb.opts_default(ir_max_sweeps=1, ir_tol=1e-300))
    assert e.value.name == "E_NOCONV"


def test_bad_arguments(fz):
    fosb, ctx, torch = fz
    m1 = fosb.Mesh(ctx, *workloads.icosphere(1))
    m2 = fosb.Mesh(ctx, *workloads.icosphere(2))
    print("[gpu] argument validation", flush=True)
    # leading dimension shorter than N
    from paper_2308_01457_amd.fosb import _P, C, lib
    Zs = torch.empty((m1.n_edges, m1.n_edges), dtype=torch.complex128, device=ctx.torch_device)
    st = lib().fosb_assemble(ctx.h, m1.h, 1.0, None, C.c_void_p(Zs.data_ptr()), m1.n_edges - 1)
    assert fosb.STATUS[st] == "E_WORKSPACE"
    # non-positive wavenumber
    with pytest.raises(fosb.FosbError) as e:
        fosb.assemble(ctx, m1, 0.0)
    assert e.value.name == "E_INVALID"
    l1 = fosb.Level(ctx, m1, 1.0, fosb.assemble(ctx, m1, 1.0), fosb.FP64)
    l2 = fosb.Level(ctx, m2, 1.0, fosb.assemble(ctx, m2, 1.0), fosb.FP64)
    # incidence index out of range
    with pytest.raises(fosb.FosbError) as e:
        fosb.rhs_correlation(ctx, l2, l1, fosb.make_cov("gaussian", 0.01, 0.5), dir=3)
    assert e.value.name == "E_INVALID"
    # correlation length must be positive for the Gaussian
    with pytest.raises(fosb.FosbError) as e:
        fosb.rhs_correlation(ctx, l2, l1, fosb.make_cov("gaussian", 0.01, 0.0))
    assert e.value.name == "E_INVALID"
    # a level of a different wavenumber in the same ladder
    l3 = fosb.Level(ctx, m1, 2.0, fosb.assemble(ctx, m1, 2.0), fosb.FP64)
    with pytest.raises(fosb.FosbError) as e:
        fosb.correlation(ctx, [l3, l2], 1, 2, fosb.make_cov("gaussian", 0.01, 0.5))
    assert e.value.name == "E_INVALID"
    # a handle of another context
    ctx2 = fosb.Context(0)
    with pytest.raises(fosb.FosbError) as e:
        fosb.two_sided_solve(ctx2, l2, l1, torch.zeros((l2.n, l1.n), dtype=torch.complex128,
                                                       device=ctx.torch_device))
    assert e.value.name == "E_INVALID"
    # device index out of range
    h = _P()
    st = lib().fosb_context_create(64, None, C.byref(h))
    assert fosb.STATUS[st] == "E_INVALID"
    assert "out of range" in lib().fosb_last_error().decode()
    # everything still works afterwards
    blocks = fosb.correlation(ctx, [l1, l2], 1, 2, fosb.make_cov("gaussian", 0.01, 0.5))
    var = fosb.far_field_moments(ctx, [l1, l2], 1, 2, blocks, workloads.angles_xz(9))
    assert np.isfinite(var.cpu().numpy()).all()


def test_handles_outlive_their_context(fz):
    """Destroying a context before its meshes and levels detaches them: a
    detached handle is rejected by every call and destroying it only frees it."""
    fosb, ctx, torch = fz
    c2 = fosb.Context(0)
    m = fosb.Mesh(c2, *workloads.icosphere(1))
    lv = fosb.Level(c2, m, 1.0, fosb.assemble(c2, m, 1.0), fosb.FP64)
    print("[gpu] context destroyed before its level and mesh", flush=True)
    c2.close()
    with pytest.raises(fosb.FosbError) as e:                  # detached level on a live context
        fosb.correlation(ctx, [lv], 1, 1, fosb.make_cov("gaussian", 0.01, 0.5))
    assert e.value.name == "E_INVALID"
    lv.close()
    m.close()
    # the other context is unaffected
    m2 = fosb.Mesh(ctx, *workloads.icosphere(1))
    assert torch.isfinite(fosb.assemble(ctx, m2, 1.0).abs()).all()


def test_phase_range_is_enforced(fz):
    """The assembly's sin/cos is exact to an ulp for phases k |x - y| up to 1e5;
    k times the mesh's bounding-box diagonal beyond that is rejected."""
    fosb, ctx, torch = fz
    m = fosb.Mesh(ctx, *workloads.icosphere(1))      # unit sphere: diagonal 2 sqrt(3) at most
    print("[gpu] wavenumber beyond the phase range", flush=True)
    with pytest.raises(fosb.FosbError) as e:
        fosb.assemble(ctx, m, 1.0e5)
    assert e.value.name == "E_INVALID"
    assert "bounding-box" in fosb.lib().fosb_last_error().decode()
    assert torch.isfinite(fosb.assemble(ctx, m, 1.0e4).abs()).all()


def test_dielectric_argument_errors(fz):
    """The dielectric entry points reject bad materials, mixed formulations and
    requests that need data the levels do not have, with the context usable."""
    fosb, ctx, torch = fz
    m = fosb.Mesh(ctx, *workloads.icosphere(1))
    n2 = 2 * m.n_edges
    print("[gpu] dielectric argument errors", flush=True)
    for eps, mu in ((0.0, 1.0), (-2.0, 1.0), (2.0, float("nan"))):
        with pytest.raises(fosb.FosbError) as e:
            fosb.assemble_pmchwt(ctx, m, 3.0, eps, mu)
        assert e.value.name == "E_INVALID"
    Zs = torch.empty((n2, n2 - 1), dtype=torch.complex128, device=ctx.torch_device)
    with pytest.raises(fosb.FosbError) as e:
        fosb.assemble_pmchwt(ctx, m, 3.0, 2.1, 1.0, Z=Zs)
    assert e.value.name == "E_WORKSPACE"
    # shape-derivative weights are built for a non-magnetic interior only
    Z = fosb.assemble_pmchwt(ctx, m, 3.0, 2.1, 1.5)
    with pytest.raises(fosb.FosbError) as e:
        fosb.Level.pmchwt(ctx, m, 3.0, 2.1, 1.5, Z, fosb.FP64, field="radial")
    assert e.value.name == "E_UNSUPPORTED"
    # levels without weights: no covariance right-hand side, no low-rank route
    Z = fosb.assemble_pmchwt(ctx, m, 3.0, 2.1, 1.0)
    lv = fosb.Level.pmchwt(ctx, m, 3.0, 2.1, 1.0, Z, fosb.FP64)
    cov = fosb.make_cov("gaussian", 0.01, 0.5)
    for call in (lambda: fosb.rhs_correlation(ctx, lv, lv, cov),
                 lambda: fosb.LowRank(ctx, [lv], cov, 100, 1e-8)):
        with pytest.raises(fosb.FosbError) as e:
            call()
        assert e.value.name == "E_INVALID"
    with pytest.raises(fosb.FosbError) as e:
        lv.sd_weights(0)
    assert e.value.name == "E_INVALID"
    # PEC-only entry points
    with pytest.raises(fosb.FosbError) as e:
        fosb.near_field_matrix(ctx, lv, np.array([[0.0, 0.0, 2.0]]))
    assert e.value.name == "E_UNSUPPORTED"
    # an EFIE level and a dielectric level do not pair; an EFIE level needs a covariance
    Ze = fosb.assemble(ctx, m, 3.0)
    le = fosb.Level(ctx, m, 3.0, Ze, fosb.FP64)
    C = torch.empty((lv.n, le.n), dtype=torch.complex128, device=ctx.torch_device)
    with pytest.raises(fosb.FosbError) as e:
        fosb.two_sided_solve(ctx, lv, le, C)
    assert e.value.name == "E_INVALID"
    with pytest.raises(fosb.FosbError) as e:
        fosb.rhs_correlation(ctx, le, le, None)
    assert e.value.name == "E_INVALID"
    # still usable: the rank-one right-hand side of the dielectric level
    C1 = fosb.rhs_correlation(ctx, lv, lv, None)
    assert torch.isfinite(C1.abs()).all()
