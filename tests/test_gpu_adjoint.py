"""GPU adjoint of the far-field variance in the covariance parameters.

* Adjoint solves X = Z^{-H} B (FP64 and mixed) on ragged sizes: backward error
  at rounding level and agreement with LAPACK.
* dS/dsigma, dS/dell and the adjoint-route S on the plain FP64 workload (unit
  icosphere s=1..3, k=1, L0=1, L=3, 181 angles) against the oracle's adjoint
  gradient, with unit and random upstream weights, Gaussian and Matern-3/2
  covariances; FP64 to 1e-10, mixed to 1e-5.
* The torch.autograd route gives the same gradient.
* At the differentiated workload's full size (s=1..4, k=3, L0=1, L=4, 91
  angles), where the oracle is too slow: dS/dell against a central difference
  (h = 1e-5) of the GPU FP64 forward pass, dS/dsigma = 2 S/sigma, S = sum V, and
  the mixed path against the FP64 path."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K1 = 1.0
SIG, ELL = 0.01, 0.5


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def fz():
    import torch
    from paper_2308_01457_amd import fosb
    assert torch.cuda.is_available()
    return fosb, fosb.Context(0), torch


def _levels(fosb, ctx, ladder, k, precision, opts=None):
    out = []
    for V, F in ladder:
        m = fosb.Mesh(ctx, V, F)
        Z = fosb.assemble(ctx, m, k)
        out.append(fosb.Level(ctx, m, k, Z, precision, opts=opts))
    return out


@pytest.fixture(scope="module")
def plain_levels(fz):
    fosb, ctx, torch = fz
    ladder = [workloads.icosphere(s) for s in (1, 2, 3)]
    print("[gpu] plain levels s=1..3 fp64 + mixed", flush=True)
    return {"fp64": _levels(fosb, ctx, ladder, K1, fosb.FP64),
            "mixed": _levels(fosb, ctx, ladder, K1, fosb.MIXED)}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_solve_backward_error(fz, precision):
    fosb, ctx, torch = fz
    rng = np.random.default_rng(11)
    for s, nrhs in ((1, 7), (2, 33), (3, 1), (3, 45)):
        V, F = workloads.icosphere(s)
        m = fosb.Mesh(ctx, V, F)
        Z = fosb.assemble(ctx, m, K1)
        Zc = Z.clone().cpu().numpy()
        prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
        print(f"[gpu] adjoint solve {precision} s={s} nrhs={nrhs}", flush=True)
        lv = fosb.Level(ctx, m, K1, Z, prec, opts=fosb.opts_default(ir_tol=1e-13))  # refine to the FP64 floor
        B = rng.standard_normal((m.n_edges, nrhs)) + 1j * rng.standard_normal((m.n_edges, nrhs))
        X = lv.solve_adjoint(torch.tensor(B, device=ctx.torch_device)).cpu().numpy()
        ZH = Zc.conj().T
        bwd = np.linalg.norm(ZH @ X - B) / (np.linalg.norm(Zc, 2) * np.linalg.norm(X))
        fwd = _rel(X, np.linalg.solve(ZH, B))
        print(f"[gpu]   backward {bwd:.2e} forward {fwd:.2e}", flush=True)
        assert bwd < 1e-14
        assert fwd < 1e-9


@pytest.mark.parametrize("precision,kind,weighted", [("fp64", "gaussian", False), ("fp64", "matern32", True),
                                                     ("mixed", "gaussian", True)])
def test_gradient_matches_oracle(fz, plain_levels, oracle_levels, precision, kind, weighted):
    fosb, ctx, torch = fz
    from oracle import uq
    n_a = 181
    xh = workloads.angles_xz(n_a)
    g = np.random.default_rng(7).standard_normal((3, n_a)) if weighted else np.ones((3, n_a))
    levels = plain_levels[precision]
    cov = fosb.make_cov(kind, SIG, ELL)
    print(f"[gpu] backward {precision} {kind} weighted={weighted}", flush=True)
    out = fosb.far_field_moments_backward(ctx, levels, 1, 3, cov, xh, torch.tensor(g, device=ctx.torch_device))
    dsig, dell, S = out.cpu().numpy()
    blocks = fosb.correlation(ctx, levels, 1, 3, cov)
    var = fosb.far_field_moments(ctx, levels, 1, 3, blocks, xh).cpu().numpy()
    olv = {s: oracle_levels(s) for s in (1, 2, 3)}
    So, go = uq.summed_variance_and_gradient(olv, 1, 3, kind, SIG, ELL, xh, weights=g)
    tol = 1e-10 if precision == "fp64" else 1e-5
    print(f"[gpu]   S {S:.6e} vs {So:.6e}; dsigma {dsig:.6e} vs {go[0]:.6e}; dell {dell:.6e} vs {go[1]:.6e}",
          flush=True)
    assert abs(S - np.sum(g * var)) < 1e-10 * np.sum(np.abs(g * var))   # adjoint route = Sigma route
    assert abs(S - So) < tol * abs(So)
    assert abs(dsig - go[0]) < tol * abs(go[0])
    assert abs(dell - go[1]) < tol * abs(go[1])


def test_autograd_function(fz, plain_levels):
    fosb, ctx, torch = fz
    n_a = 37
    xh = workloads.angles_xz(n_a)
    levels = plain_levels["fp64"]
    g = torch.tensor(np.random.default_rng(2).standard_normal((3, n_a)), device=ctx.torch_device)
    sigma = torch.tensor(SIG, dtype=torch.float64, requires_grad=True)
    ell = torch.tensor(ELL, dtype=torch.float64, requires_grad=True)
    print("[gpu] autograd backward", flush=True)
    var = fosb.rcs_variance(ctx, levels, 1, 3, "gaussian", sigma, ell, xh)
    loss = (g * var).sum()
    loss.backward()
    ref = fosb.far_field_moments_backward(ctx, levels, 1, 3, fosb.make_cov("gaussian", SIG, ELL), xh, g).cpu()
    assert abs(sigma.grad.item() - ref[0].item()) <= 1e-14 * abs(ref[0].item())
    assert abs(ell.grad.item() - ref[1].item()) <= 1e-14 * abs(ref[1].item())
    assert abs(loss.item() - ref[2].item()) < 1e-10 * abs(ref[2].item())


def test_gradient_full_size_finite_difference(fz):
    """Differentiated workload: unit icosphere s=1..4 (N up to 7680), k=3,
    Gaussian radial covariance (0.01, 0.5), L0=1, L=4, 91 angles."""
    fosb, ctx, torch = fz
    w = workloads.workload("grad_k3")
    xh = w.angles
    ones = torch.ones((3, w.n_angles), dtype=torch.float64, device=ctx.torch_device)
    print("[gpu] grad_k3 fp64 levels s=1..4", flush=True)
    lv64 = _levels(fosb, ctx, w.meshes, w.k, fosb.FP64)

    def S_of(ell, levels):
        cov = fosb.make_cov(w.cov_kind, w.sigma, ell)
        blocks = fosb.correlation(ctx, levels, w.L0, w.L, cov)
        return float(fosb.far_field_moments(ctx, levels, w.L0, w.L, blocks, xh).sum().item())

    cov = fosb.make_cov(w.cov_kind, w.sigma, w.ell)
    dsig, dell, S = fosb.far_field_moments_backward(ctx, lv64, w.L0, w.L, cov, xh, ones).cpu().numpy()
    S0 = S_of(w.ell, lv64)
    h = 1e-5
    fd = (S_of(w.ell + h, lv64) - S_of(w.ell - h, lv64)) / (2 * h)
    print(f"[gpu]   S {S:.8e} (forward {S0:.8e}); dell {dell:.8e} fd {fd:.8e}; dsigma {dsig:.8e}", flush=True)
    assert abs(S - S0) < 1e-10 * abs(S0)
    assert abs(dsig - 2 * S / w.sigma) < 1e-12 * abs(dsig)
    assert abs(dell - fd) < 1e-6 * abs(dell)
    del lv64
    print("[gpu] grad_k3 mixed levels s=1..4", flush=True)
    lv32 = _levels(fosb, ctx, w.meshes, w.k, fosb.MIXED)
    g32 = fosb.far_field_moments_backward(ctx, lv32, w.L0, w.L, cov, xh, ones).cpu().numpy()
    print(f"[gpu]   mixed dsigma {g32[0]:.8e} dell {g32[1]:.8e}", flush=True)
    assert abs(g32[0] - dsig) < 1e-5 * abs(dsig)
    assert abs(g32[1] - dell) < 1e-5 * abs(dell)


def test_gradient_full_size_against_oracle_golden(fz):
    """Differentiated workload (s = 1..4, k = 3, L0 = 1, L = 4, 91 angles)
    against tests/golden/grad_k3_oracle.json, written by
    make_grad_k3_golden.py from the FP64 oracle alone: S, dS/dsigma and
    dS/dell to 1e-6 (FP64 path) and 1e-5 (mixed path), and the variance."""
    fosb, ctx, torch = fz
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grad_k3_oracle.json")) as f:
        gold = json.load(f)
    w = workloads.workload("grad_k3")
    xh = w.angles
    Vo = np.asarray(gold["variance"])
    ones = torch.ones((3, w.n_angles), dtype=torch.float64, device=ctx.torch_device)
    cov = fosb.make_cov(w.cov_kind, w.sigma, w.ell)
    for prec, name, tol in ((fosb.FP64, "fp64", 1e-6), (fosb.MIXED, "mixed", 1e-5)):
        print(f"[gpu] grad_k3 {name} against the oracle golden", flush=True)
        lv = _levels(fosb, ctx, w.meshes, w.k, prec)
        blocks = fosb.correlation(ctx, lv, w.L0, w.L, cov)
        var = fosb.far_field_moments(ctx, lv, w.L0, w.L, blocks, xh).cpu().numpy()
        del blocks
        dsig, dell, S = fosb.far_field_moments_backward(ctx, lv, w.L0, w.L, cov, xh, ones).cpu().numpy()
        ev = float(np.linalg.norm(var - Vo) / np.linalg.norm(Vo))
        es = abs(S - gold["S"]) / abs(gold["S"])
        eg = max(abs(dsig - gold["dS_dsigma"]) / abs(gold["dS_dsigma"]), abs(dell - gold["dS_dell"]) / abs(gold["dS_dell"]))
        print(f"[gpu]   variance {ev:.2e}  S {es:.2e}  gradient {eg:.2e}", flush=True)
        assert ev < tol and es < tol and eg < tol
        del lv
