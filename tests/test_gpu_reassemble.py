"""MIXED levels that keep no complex128 copy of Z (Z = NULL): Zlow assembled
in FP64 column bands and rounded, and every refinement residual computed with
Z re-assembled band by band.  Against levels with the stored FP64 matrix on
the superquadric ladder (k = 8, s = 3, 4): refined solves, first moments and
the whole pass (fosb_second_moment with the finest level re-assembling)."""

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


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_reassembled_level_solves_match_stored(fz):
    fosb, ctx, torch = fz
    k = 8.0
    m = fosb.Mesh(ctx, *workloads.superquadric(3))
    opts = fosb.opts_default(ir_tol=1e-13, ir_max_sweeps=20)
    print("[gpu] re-assembled level, superquadric s=3, k=8", flush=True)
    Z = fosb.assemble(ctx, m, k, opts)
    ref = fosb.Level(ctx, m, k, Z, fosb.MIXED, opts=opts)
    lv = fosb.Level(ctx, m, k, None, fosb.MIXED, opts=opts)
    e_u = _rel(lv.first_moment().cpu().numpy(), ref.first_moment().cpu().numpy())
    rng = np.random.default_rng(3)
    B = torch.tensor(rng.standard_normal((m.n_edges, 8)) + 1j * rng.standard_normal((m.n_edges, 8)),
                     device=ctx.torch_device)
    st = fosb.Stats()
    X = lv.solve(B.clone(), st).cpu().numpy()
    Xr = ref.solve(B.clone()).cpu().numpy()
    e_x = _rel(X, Xr)
    Zh, Bh = Z.cpu().numpy(), B.cpu().numpy()
    res = np.linalg.norm(Bh - Zh @ X) / (np.linalg.norm(Zh) * np.linalg.norm(X))
    print(f"[gpu]   first moment {e_u:.2e}, solve {e_x:.2e}, backward error {res:.2e}, sweeps {st.ir_sweeps}",
          flush=True)
    assert e_u < 1e-11 and e_x < 1e-11 and res < 1e-14
    with pytest.raises(fosb.FosbError) as e:
        lv.solve_adjoint(B.clone())
    assert e.value.name == "E_UNSUPPORTED"


def test_reassembled_finest_level_in_the_pass(fz):
    fosb, ctx, torch = fz
    w = workloads.workload("superquad_k8", max_level=4)
    xh = workloads.angles_xz(91)
    cov = fosb.make_cov(w.cov_kind, w.sigma, w.ell)
    meshes = [fosb.Mesh(ctx, V, F) for V, F in w.meshes]
    opts = fosb.opts_default(ir_tol=1e-12)
    dev = ctx.torch_device
    Z = [torch.empty((m.n_edges, m.n_edges), dtype=torch.complex128, device=dev) for m in meshes]
    print("[gpu] pass with a re-assembled finest level, superquadric s=3..4", flush=True)
    v_ref, _, _ = fosb.second_moment(ctx, meshes, w.L0, w.L, w.k, fosb.MIXED, cov, xh, opts=opts, Z=Z)
    Z[-1] = None
    v, _, _ = fosb.second_moment(ctx, meshes, w.L0, w.L, w.k, fosb.MIXED, cov, xh, opts=opts, Z=Z)
    v64, _, _ = fosb.second_moment(ctx, meshes, w.L0, w.L, w.k, fosb.FP64, cov, xh)
    e, e64 = _rel(v.cpu().numpy(), v_ref.cpu().numpy()), _rel(v.cpu().numpy(), v64.cpu().numpy())
    print(f"[gpu]   variance vs stored-Z mixed {e:.2e}, vs FP64 {e64:.2e}", flush=True)
    assert e < 1e-9 and e64 < 1e-9


def test_reassembled_level_certificate(fz):
    """opts.certify on a level without the FP64 matrix: the condition estimate
    (from the unrefined FP32 factors) and the growth factor agree with the
    stored-matrix level's, and refined solves report an FP64 backward error
    below 1e-13 from the re-assembled residual."""
    fosb, ctx, torch = fz
    k = 8.0
    m = fosb.Mesh(ctx, *workloads.superquadric(3))
    opts = fosb.opts_default(ir_tol=1e-13, ir_max_sweeps=20, certify=1)
    ref = fosb.Level(ctx, m, k, fosb.assemble(ctx, m, k, opts), fosb.MIXED, opts=opts)
    lv = fosb.Level(ctx, m, k, None, fosb.MIXED, opts=opts)
    (k_ref, g_ref), (k_re, g_re) = ref.certificate(), lv.certificate()
    B = torch.tensor(np.random.default_rng(4).standard_normal((m.n_edges, 4)) + 0j, device=ctx.torch_device)
    st = fosb.Stats()
    lv.solve(B, st)
    print(f"[gpu] re-assembled certificate: kappa1 {k_re:.6e} ({k_ref:.6e}), growth {g_re:.6e} ({g_ref:.6e}), "
          f"backward error {st.backward_error:.2e}", flush=True)
    assert abs(k_re - k_ref) < 1e-3 * k_ref and abs(g_re - g_ref) < 1e-5 * g_ref
    assert 0 < st.backward_error < 1e-13
